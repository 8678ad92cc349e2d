// Level stepping of one EMT case for partition trees whose coupling levels do not fit every
// workgroup's LDS (paper Section II, Eq. (1)-(2); coupling levels of Section III.B made exact;
// line changes as the SMW correction standing in for Section IV's update).
//
// One workgroup per leaf of the tree, all steps in one cooperative launch.  A workgroup owns the
// rows of its leaf, the coupling columns whose endpoint row it owns, and those columns' rows of
// their node's S_t^{-1}.  Per apply:
//   1. v = B_l^{-1} x on the own rows (GEMV from LDS);
//   2. for every level, bottom-up: the owners publish s_g = sqrt|G_ab| v[row_g] (own rows are
//      already corrected through the levels below); barrier; the owners publish
//      y_g = (S_t^{-1} s)_g; barrier; every workgroup subtracts its rows of Z_t y_t;
//   3. the own rows' values are published; barrier; every workgroup reads its X rows
//      (neighbours through G, line-loss endpoints) and applies the active line changes' SMW
//      correction to own rows and X rows with the same operations, so shared rows agree bitwise.
// Each exchanged value has exactly one writer, so no row is computed twice.  FP32 storage refines
// against the FP64 residual; FP64 storage warm-started runs the incremental form
// v = v_prev + P (b - G v_prev), one apply per step.
#include "hinv_internal.h"
#include "team_sync.h"

namespace hinv {

constexpr int kLThreads = 1024;
constexpr int kLWaves = kLThreads / 64;
static_assert(HINV_MAX_LEAF * 8 <= kLThreads, "leaf GEMV: one row per group of eight lanes");

template <typename TB>
struct LAcc { using T = float; };
template <>
struct LAcc<double> { using T = double; };

struct LevelLayout {
    size_t blk, zown, srow, uown, ux;
    size_t b, v, t, d, xv, xd, yl, h0, h1, hC, gC, oval, bg, bal, samp, sph, sn, ocw, cinv, mdg, red, tz;
    size_t optr, ocl, orow, osoff, oc0, om, xrow, ozo, opm, opc, orp, ocol, bglob, bf, bt, iptr, ibr, sptr;
    size_t lpa, lpb, mact, lbr, lst, vg, ctl;
    size_t total;
};

template <typename TB, bool MIXED>
__host__ __device__ inline LevelLayout level_layout(const LevelDev& D, int R)
{
    LevelLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = (o + bytes + 15) & ~(size_t)15;
        return r;
    };
    const size_t NL = D.NL, NX = D.NX, NB = D.NB, H = D.H, NO = D.NO;
    const size_t S = sizeof(TB), F = sizeof(double), I = sizeof(int);
    L.blk = take(S * NL * NL);
    L.zown = take(S * D.ZO);
    L.srow = take(S * D.SO);
    L.uown = take(S * R * NL);
    L.ux = take(S * R * NX);
    L.b = take(F * NL);
    L.v = take(F * NL);
    L.t = take(MIXED ? F * NL : 0);
    L.d = take(MIXED ? F * NL : 0);
    L.xv = take(F * NX);
    L.xd = take(MIXED ? F * NX : 0);
    L.yl = take(F * D.PM);
    L.h0 = take(F * NB);
    L.h1 = take(F * NB);
    L.hC = take(F * NL);
    L.gC = take(F * NL);
    L.oval = take(MIXED ? F * D.NE : 0);
    L.bg = take(F * NB);
    L.bal = take(F * NB);
    L.samp = take(F * D.NS);
    L.sph = take(F * D.NS);
    L.sn = take(F * D.NS);
    L.ocw = take(F * NO);
    L.cinv = take(F * R * R * R);
    L.mdg = take(F * R);
    L.red = take(F * 2 * kLWaves);
    L.tz = take(F * 2 * R);
    L.optr = take(I * (H + 1));
    L.ocl = take(I * NO);
    L.orow = take(I * NO);
    L.osoff = take(I * NO);
    L.oc0 = take(I * NO);
    L.om = take(I * NO);
    L.xrow = take(I * NX);
    L.ozo = take(I * H);
    L.opm = take(I * H);
    L.opc = take(I * H);
    L.orp = take(I * (NL + 1));
    L.ocol = take(MIXED ? I * D.NE : 0);
    L.bglob = take(I * NB);
    L.bf = take(I * NB);
    L.bt = take(I * NB);
    L.iptr = take(I * (NL + 1));
    L.ibr = take(I * D.NI);
    L.sptr = take(I * (NL + 1));
    L.lpa = take(I * R);
    L.lpb = take(I * R);
    L.mact = take(I * R);
    L.lbr = take(I * R);
    L.lst = take(I * R);
    L.vg = take(sizeof(unsigned long long));
    L.ctl = take(I * 8);
    L.total = o;
    return L;
}

size_t level_lds_bytes(const LevelDev& D, int R, int prec, int warm)
{
    if (prec != HINV_FP64) return level_layout<float, true>(D, R).total;
    return warm ? level_layout<double, true>(D, R).total : level_layout<double, false>(D, R).total;
}

// The stepping of one case by its T workgroups (w = this workgroup's leaf).  Ld gives the LDS
// layout (the case's own dimensions, or the maxima over the cases of one launch); D the case's
// tables; step0 the first step of the launch.
template <typename TB, bool MIXED, bool WARM>
__device__ void level_body(const LevelDev& Ld, const LevelDev& D, const EmtDev& E, const HierDev& H, const ModDev& M,
                           const RunParams& P, int64_t step0, int w, unsigned char* L8)
{
    using TA = typename LAcc<TB>::T;
    // MIXED with FP64 storage is the incremental form v = v_prev + P (b - G v_prev): one FP64 apply of
    // the residual per step, no convergence statistics
    constexpr bool INC = MIXED && sizeof(TB) == 8;
    static_assert(!INC || WARM, "the incremental FP64 form starts from the previous step's voltages");
    const int R = M.R;
    const LevelLayout Ly = level_layout<TB, MIXED>(Ld, R);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform in the wavefront
    const int n = H.n, NL = Ld.NL, NX = Ld.NX, Hn = D.H, T = D.T;
    const int lo = D.w_lo[w], nl = D.w_nl[w], nx = D.w_nx[w], nb = D.w_nb[w];
    TB* blk = (TB*)(L8 + Ly.blk);
    TB* zown = (TB*)(L8 + Ly.zown);
    TB* srow = (TB*)(L8 + Ly.srow);
    TB* uown = (TB*)(L8 + Ly.uown);
    TB* ux = (TB*)(L8 + Ly.ux);
    double* b = (double*)(L8 + Ly.b);
    double* v = (double*)(L8 + Ly.v);
    double* t = (double*)(L8 + Ly.t);
    double* d = (double*)(L8 + Ly.d);
    double* xv = (double*)(L8 + Ly.xv);
    double* xd = (double*)(L8 + Ly.xd);
    double* yl = (double*)(L8 + Ly.yl);
    double* hc = (double*)(L8 + Ly.h0);
    double* hn = (double*)(L8 + Ly.h1);
    double* hC = (double*)(L8 + Ly.hC);
    double* gC = (double*)(L8 + Ly.gC);
    double* oval = (double*)(L8 + Ly.oval);
    double* bg = (double*)(L8 + Ly.bg);
    double* bal = (double*)(L8 + Ly.bal);
    double* samp = (double*)(L8 + Ly.samp);
    double* sph = (double*)(L8 + Ly.sph);
    double* sn = (double*)(L8 + Ly.sn);
    double* ocw = (double*)(L8 + Ly.ocw);
    double* cinv = (double*)(L8 + Ly.cinv);
    double* mdg = (double*)(L8 + Ly.mdg);
    double* red = (double*)(L8 + Ly.red);
    double* tz = (double*)(L8 + Ly.tz);
    int* optr = (int*)(L8 + Ly.optr);
    int* ocl = (int*)(L8 + Ly.ocl);
    int* orow = (int*)(L8 + Ly.orow);
    int* osoff = (int*)(L8 + Ly.osoff);
    int* oc0 = (int*)(L8 + Ly.oc0);
    int* om = (int*)(L8 + Ly.om);
    int* xrow = (int*)(L8 + Ly.xrow);
    int* ozo = (int*)(L8 + Ly.ozo);
    int* opm = (int*)(L8 + Ly.opm);
    int* opc = (int*)(L8 + Ly.opc);
    int* orp = (int*)(L8 + Ly.orp);
    int* ocol = (int*)(L8 + Ly.ocol);
    int* bglob = (int*)(L8 + Ly.bglob);
    int* bf = (int*)(L8 + Ly.bf);
    int* bt = (int*)(L8 + Ly.bt);
    int* iptr = (int*)(L8 + Ly.iptr);
    int* ibr = (int*)(L8 + Ly.ibr);
    int* sptr = (int*)(L8 + Ly.sptr);
    int* lpa = (int*)(L8 + Ly.lpa);
    int* lpb = (int*)(L8 + Ly.lpb);
    int* mact = (int*)(L8 + Ly.mact);
    int* lbr = (int*)(L8 + Ly.lbr);
    int* lst = (int*)(L8 + Ly.lst);
    unsigned long long* vg = (unsigned long long*)(L8 + Ly.vg);
    int* ctl = (int*)(L8 + Ly.ctl);

    const TB* gblk;
    const TB* gS;
    const TB* gZ;
    const TB* gU;
    if constexpr (sizeof(TB) == 8) {
        gblk = (const TB*)H.blk; gS = (const TB*)H.Sinv; gZ = (const TB*)H.Z; gU = (const TB*)M.U;
    } else {
        gblk = (const TB*)H.blk32; gS = (const TB*)H.Sinv32; gZ = (const TB*)H.Z32; gU = (const TB*)M.U32;
    }
    // ---------------- tables and state into LDS
    {
        const TB* src = gblk + H.leaf_off[w];
        for (int i = tid; i < nl * nl; i += kLThreads) blk[i] = src[i];
        const int* wop = D.optr + (int64_t)w * (Hn + 1);
        for (int hh = tid; hh <= Hn; hh += kLThreads) optr[hh] = wop[hh];
        const int no = wop[Hn];
        for (int k = tid; k < no; k += kLThreads) {          // owned columns and their rows of S^{-1}
            const int64_t gk = (int64_t)w * D.NO + k;
            const int g = D.ocl[gk], node = H.col_node[g];
            const int m = H.node_m[node], q = g - H.node_col0[node];
            ocl[k] = g;
            orow[k] = D.orow[gk];
            osoff[k] = D.osoff[gk];
            oc0[k] = H.node_col0[node];
            om[k] = m;
            ocw[k] = H.col_w[g];
            const TB* s0 = gS + H.node_soff[node] + q;
            TB* dst = srow + D.osoff[gk];
            for (int p = 0; p < m; ++p) dst[p] = s0[(int64_t)p * m];
        }
        for (int hh = 0; hh < Hn; ++hh) {                      // own rows: Z panel rows at every level
            const int zo = D.ozo[w * Hn + hh];
            if (tid == 0) { ozo[hh] = zo; opm[hh] = D.opm[w * Hn + hh]; opc[hh] = D.opc[w * Hn + hh]; }
            if (zo >= 0) {
                const int pan = D.opan[w * Hn + hh], pm = D.opm[w * Hn + hh];
                const TB* zp = gZ + H.pan_zoff[pan] + (lo - H.pan_lo[pan]);
                for (int i = tid; i < pm * nl; i += kLThreads) {
                    const int j = i / nl, r = i - j * nl;
                    zown[zo + i] = zp[(int64_t)j * H.pan_n[pan] + r];
                }
            }
        }
        const int* wx = D.xrow + (int64_t)w * D.NX;
        for (int x = tid; x < nx; x += kLThreads) xrow[x] = wx[x];
        const int64_t rb = (int64_t)w * (D.NL + 1);
        for (int r = tid; r <= nl; r += kLThreads) {
            orp[r] = D.orp[rb + r];
            iptr[r] = D.iptr[rb + r];
            sptr[r] = D.sptr[rb + r];
        }
        if (MIXED) {
            for (int e = tid; e < D.orp[rb + nl]; e += kLThreads) {
                ocol[e] = D.ocol[(int64_t)w * D.NE + e];
                oval[e] = D.oval[(int64_t)w * D.NE + e];
            }
        }
        for (int i = tid; i < D.iptr[rb + nl]; i += kLThreads) ibr[i] = D.ibr[(int64_t)w * D.NI + i];
        for (int i = tid; i < D.sptr[rb + nl]; i += kLThreads) {
            samp[i] = D.samp[(int64_t)w * D.NS + i];
            sph[i] = D.sph[(int64_t)w * D.NS + i];
        }
        for (int q = tid; q < nb; q += kLThreads) {
            const int64_t gq = (int64_t)w * D.NB + q;
            bglob[q] = D.bglob[gq];
            bf[q] = D.bf[gq];
            bt[q] = D.bt[gq];
            bg[q] = D.bg[gq];
            bal[q] = D.bal[gq];
            hc[q] = E.h[(int64_t)(step0 & 1) * E.n_cases * E.nbr + D.bglob[gq]];
        }
        for (int r = tid; r < nl; r += kLThreads) {
            b[r] = E.b[lo + r];
            v[r] = E.v[lo + r];
            hC[r] = E.hC[lo + r];
            gC[r] = E.gC[lo + r];
        }
        for (int x = tid; x < nx; x += kLThreads) xv[x] = E.v[wx[x]];
        const int cnt = M.count[0];
        if (tid == 0) {
            ctl[1] = cnt;
            ctl[2] = E.loss_cnt[0];
        }
        if (tid < R) {
            mact[tid] = tid < cnt ? M.act[tid] : 0x7fffffff;
            mdg[tid] = M.dg[tid];
            lpa[tid] = D.lpa[(int64_t)w * R + tid];
            lpb[tid] = D.lpb[(int64_t)w * R + tid];
            lbr[tid] = E.loss_br[tid];
            lst[tid] = E.loss_step[tid];
            if (tid < cnt && (D.lpa[(int64_t)w * R + tid] < 0 || (M.b[tid] >= 0 && D.lpb[(int64_t)w * R + tid] < 0)))
                atomicOr(P.flags, kFlagTeamRow);
        }
        for (int i = tid; i < R * R * R; i += kLThreads) cinv[i] = M.Cinv[i];
        for (int i = tid; i < R * nl; i += kLThreads) {
            const int j = i / nl, r = i - j * nl;
            uown[j * NL + r] = j < cnt ? gU[(int64_t)j * n + lo + r] : (TB)0;
        }
        for (int i = tid; i < R * nx; i += kLThreads) {
            const int j = i / nx, x = i - j * nx;
            ux[j * NX + x] = j < cnt ? gU[(int64_t)j * n + wx[x]] : (TB)0;
        }
    }
    __syncthreads();
    const int cnt = ctl[1], nlost = ctl[2];
    unsigned int epoch = 0;
    bool alive = true;
    double worst = 0.0;
    unsigned int* flags = D.sync;

    auto cval = [&](const double* own, const double* xr, int comb) -> double {
        return comb < nl ? own[comb] : xr[comb - nl];
    };

    // one application of the stored inverse with the active line changes:
    // out (own rows), outx (X rows) from xin (own rows)
    // tags of the y exchange: ((step + 1) * applies per step + apply of the step) * 8 + level, unique
    // over the case's run (the buffer is cleared when the tables are uploaded)
    const int64_t A = (MIXED && !INC) ? (int64_t)P.max_refine + 1 : 1;
    const int ncol = H.lvl_col[Hn];      // coupling columns of the tree
    int64_t cur_step = step0;
    int ais = 0;
    unsigned int ytag0 = 0;
    auto apply = [&](const double* xin, double* out, double* outx, int ract, bool want_vm) -> bool {
        ytag0 = (unsigned int)(((cur_step + 1) * A + ais++) * 8);
        {   // leaf product: eight lanes per row r = tid / 8, lane c takes the block columns j = c (mod 8);
            // the eight partial sums are added by DPP moves
            const int r = tid >> 3, c = tid & 7;
            const bool act = r < nl;      // whole groups of eight lanes are active or not
            TA acc = 0;
            if (act)
                for (int j = c; j < nl; j += 8) acc += (TA)blk[j * nl + r] * (TA)xin[j];
            const double val = oct_sum((double)acc);
            if (act && c == 0) out[r] = val;
        }
        __syncthreads();
        // The only barrier of an apply is the top level's s exchange (top-level s double-buffered by
        // apply parity).  The s of the lower levels, every y and the final values are tagged words:
        // every such slot is next written after the next apply has passed this apply's top-level
        // barrier (or, for top-level y and the final values, the next apply's), and every workgroup
        // reads the current value before it arrives there.
        double* Sxp = D.Sx + (int64_t)((ytag0 >> 3) & 1u) * ncol;
        for (int hl = 1; hl <= Hn; ++hl) {
            const int k0 = optr[hl - 1], k1 = optr[hl];
            const bool top = hl == Hn;
            const unsigned int ytag = ytag0 + (unsigned int)hl;
            if (top) {
                for (int k = k0 + tid; k < k1; k += kLThreads) xchg_store(&Sxp[ocl[k]], ocw[k] * out[orow[k]]);
                if (!count_barrier(flags, T, ++epoch, P.flags, ctl)) return false;
            } else {
                for (int k = k0 + tid; k < k1; k += kLThreads) tagged_store(D.SL + 2 * ocl[k], ocw[k] * out[orow[k]], ytag);
            }
            bool sok = true;
            for (int k = k0 + wave; k < k1; k += kLWaves) {   // y of the owned columns, one wavefront each
                const int m = om[k], c0 = oc0[k];
                const TB* Sr = srow + osoff[k];
                TA acc = 0;
                for (int p = lane; p < m; p += 64) {
                    const double sv = top ? xchg_load(&Sxp[c0 + p]) : tagged_load(D.SL + 2 * (c0 + p), ytag, &sok);
                    acc += (TA)Sr[p] * (TA)sv;
                }
                for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
                if (lane == 0) tagged_store(D.YL + 2 * ocl[k], (double)acc, ytag);
            }
            if (!top && __syncthreads_or(sok ? 0 : 1)) {
                if (tid == 0) atomicOr(P.flags, kFlagBarrier);
                return false;
            }
            const int zo = ozo[hl - 1];
            if (zo >= 0) {                                     // own rows: v -= Z_t y_t
                const int pm = opm[hl - 1], pc = opc[hl - 1];
                bool ok = true;
                for (int j = tid; j < pm; j += kLThreads) yl[j] = tagged_load(D.YL + 2 * (pc + j), ytag, &ok);
                if (__syncthreads_or(ok ? 0 : 1)) {
                    if (tid == 0) atomicOr(P.flags, kFlagBarrier);
                    return false;
                }
                for (int idx = tid; idx < nl * 8; idx += kLThreads) {   // eight lanes per own row
                    const int r = idx >> 3, sub = idx & 7;
                    TA acc = 0;
                    for (int j = sub; j < pm; j += 8) acc += (TA)zown[zo + j * nl + r] * (TA)yl[j];
                    acc = oct_sum(acc);
                    if (sub == 0) out[r] -= (double)acc;
                }
                __syncthreads();
            }
        }
        // the own rows' values for the X rows of other workgroups.  With two or more levels and no
        // team-wide norm to gather, they go as tagged values without a barrier: a row's next write
        // comes after the next apply's first s barrier, and its next s values (level 1) after this
        // apply's last s barrier, which every workgroup reaches after its reads of both
        if (Hn >= 2 && !want_vm) {
            for (int r = tid; r < nl; r += kLThreads) tagged_store(D.VL + 2 * (lo + r), out[r], ytag0);
            bool ok = true;
            for (int x = tid; x < nx; x += kLThreads) outx[x] = tagged_load(D.VL + 2 * xrow[x], ytag0, &ok);
            if (__syncthreads_or(ok ? 0 : 1)) {
                if (tid == 0) atomicOr(P.flags, kFlagBarrier);
                return false;
            }
        } else {
            for (int r = tid; r < nl; r += kLThreads) xchg_store(&D.V1[lo + r], out[r]);
            if (!count_barrier(flags, T, ++epoch, P.flags, ctl)) return false;
            if (want_vm) {     // the team's largest |v| (vg was cleared before this apply)
                for (int i = tid; i < T; i += kLThreads)
                    atomicMax(vg, (unsigned long long)__double_as_longlong(xchg_load(&D.VM[i])));
            }
            for (int x = tid; x < nx; x += kLThreads) outx[x] = xchg_load(&D.V1[xrow[x]]);
            __syncthreads();
        }
        if (ract > 0) {
            if (tid < ract) tz[tid] = cval(out, outx, lpa[tid]) - (lpb[tid] >= 0 ? cval(out, outx, lpb[tid]) : 0.0);
            __syncthreads();
            if (tid < ract) {
                const double* Ci = cinv + (ract - 1) * R * R;
                double acc = 0.0;
                for (int j = 0; j < ract; ++j) acc += Ci[tid * R + j] * tz[j];
                tz[R + tid] = acc;
            }
            __syncthreads();
            for (int r = tid; r < nl; r += kLThreads) {
                double acc = 0.0;
                for (int j = 0; j < ract; ++j) acc += (double)uown[j * NL + r] * tz[R + j];
                out[r] -= acc;
            }
            for (int x = tid; x < nx; x += kLThreads) {
                double acc = 0.0;
                for (int j = 0; j < ract; ++j) acc += (double)ux[j * NX + x] * tz[R + j];
                outx[x] -= acc;
            }
            __syncthreads();
        }
        return true;
    };

    // t = b - G_step v on own rows (FP64), then v += P t; stats on the last pass
    auto refine = [&](int ract, bool last) -> bool {
        for (int r = tid; r < nl; r += kLThreads) {
            double acc = 0.0;
            for (int e = orp[r]; e < orp[r + 1]; ++e) acc += oval[e] * cval(v, xv, ocol[e]);
            for (int j = 0; j < ract; ++j) {
                const int a = lpa[j], bb = lpb[j];
                if (a != r && bb != r) continue;
                const double wv = cval(v, xv, a) - (bb >= 0 ? cval(v, xv, bb) : 0.0);
                acc += (a == r ? 1.0 : -1.0) * mdg[j] * wv;
            }
            t[r] = b[r] - acc;
        }
        if (last) {        // publish this workgroup's max |v| for the team-wide norm
            double vm = 0.0;
            for (int r = tid; r < nl; r += kLThreads) vm = fmax(vm, fabs(v[r]));
            for (int o = 32; o > 0; o >>= 1) vm = fmax(vm, __shfl_xor(vm, o));
            if (lane == 0) red[kLWaves + wave] = vm;
            __syncthreads();
            if (tid == 0) {
                double V = 0.0;
                for (int q = 0; q < kLWaves; ++q) V = fmax(V, red[kLWaves + q]);
                xchg_store(&D.VM[w], V);
                *vg = 0ull;
            }
        }
        __syncthreads();
        if (!apply(t, d, xd, ract, last)) return false;
        double dm = 0.0;
        for (int r = tid; r < nl; r += kLThreads) {
            v[r] += d[r];
            dm = fmax(dm, fabs(d[r]));
        }
        for (int x = tid; x < nx; x += kLThreads) xv[x] += xd[x];
        if (last) {        // max |d| over the own rows / the team's max |v|
            for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o));
            if (lane == 0) red[wave] = dm;
            __syncthreads();
            if (tid == 0) {
                double Dm = 0.0;
                for (int q = 0; q < kLWaves; ++q) Dm = fmax(Dm, red[q]);
                const double V = __longlong_as_double((long long)*vg);
                const double ratio = V > 0.0 ? Dm / V : (Dm > 0.0 ? INFINITY : 0.0);
                if (!isfinite(ratio)) atomicOr(P.flags, kFlagNaN);
                else {
                    worst = fmax(worst, ratio);
                    if (ratio > P.rel_tol) atomicOr(P.flags, kFlagNoConv);
                }
            }
        }
        __syncthreads();
        return true;
    };

    int64_t applies = 0;
    const int ns = sptr[nl];
    for (int it = 0; it < P.n_steps && alive; ++it) {
        const int64_t step = step0 + it;
        cur_step = step;
        ais = 0;
        int ract = 0;
        while (ract < cnt && (int64_t)mact[ract] <= step) ++ract;
        if constexpr (!MIXED) {
            alive = apply(b, v, xv, ract, false);
            applies += 1;
        } else {
            const int nref = INC ? 1 : (WARM ? P.max_refine + 1 : P.max_refine);
            if (!WARM) {
                alive = apply(b, v, xv, ract, false);
                applies += 1;
            }
            for (int q = 0; q < nref && alive; ++q) {
                alive = refine(ract, !INC && q == nref - 1);
                applies += 1;
            }
        }
        if (!alive) break;
        // history: new branch histories, then the right-hand side of step+1
        for (int q = tid; q < nb; q += kLThreads) {
            const int e = bglob[q];
            bool lost = false;
            for (int j = 0; j < nlost; ++j)
                if (lbr[j] == e && (int64_t)lst[j] <= step + 1) lost = true;
            double hv = 0.0;
            if (!lost) {
                const double vft = cval(v, xv, bf[q]) - cval(v, xv, bt[q]);
                const double ie = bg[q] * vft + hc[q];
                hv = bg[q] * vft + bal[q] * ie;
            }
            hn[q] = hv;
        }
        if (tid >= kLThreads - 64) {      // source injections of step+1, by the last wavefront
            for (int q = tid - (kLThreads - 64); q < ns; q += 64)
                sn[q] = samp[q] * sin(E.omega * ((double)(step + 1) * E.dt) + sph[q]);
        }
        __syncthreads();
        const int64_t jr = step - P.rec_step0;
        const bool rec = jr >= 0 && jr < P.rec_cap;
        for (int r = tid; r < nl; r += kLThreads) {
            const double va = v[r];
            double bn = 0.0;
            for (int q = sptr[r]; q < sptr[r + 1]; ++q) bn += sn[q];
            for (int q = iptr[r]; q < iptr[r + 1]; ++q) {
                const int lb = ibr[q];
                const double hv = hn[lb];
                bn -= (bf[lb] == r) ? hv : -hv;
            }
            const double ic = gC[r] * va + hC[r];
            const double hcn = -gC[r] * va - ic;
            hC[r] = hcn;
            bn -= hcn;
            if (rec) {
                const int64_t o = jr * (int64_t)n + E.perm[lo + r];
                if (P.v_rec) P.v_rec[o] = va;
                if (P.b_rec) P.b_rec[o] = b[r];
            }
            b[r] = bn;
        }
        double* tmp = hc;
        hc = hn;
        hn = tmp;
        __syncthreads();
        if (P.clk && w == 0 && tid == 0 && step - step0 < P.clk_cap)
            P.clk[step - step0] = (int64_t)wall_clock64();
    }
    if (!alive) return;
    const int64_t nstep = step0 + P.n_steps;
    for (int r = tid; r < nl; r += kLThreads) {
        E.b[lo + r] = b[r];
        E.v[lo + r] = v[r];
        E.hC[lo + r] = hC[r];
    }
    for (int q = tid; q < nb; q += kLThreads)
        if (D.bown[(int64_t)w * D.NB + q]) E.h[(int64_t)(nstep & 1) * E.n_cases * E.nbr + bglob[q]] = hc[q];
    if (tid == 0) {
        if (MIXED && !INC && P.stats) atomicMax(&P.stats[0], (unsigned long long)__double_as_longlong(worst));
        if (w == 0) {
            if (P.applies) atomicAdd(&P.applies[0], (unsigned long long)applies);
            *E.step = nstep;
        }
    }
}

template <typename TB, bool MIXED, bool WARM>
__global__ __launch_bounds__(kLThreads) void k_emt_level(LevelDev D, EmtDev E, HierDev H, ModDev M, RunParams P)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char L8[];
    level_body<TB, MIXED, WARM>(D, D, E, H, M, P, P.step0, blockIdx.x, L8);
}

// Several cases in one launch (serving): case k owns workgroups cases[k].wg0 .. + its T; the
// first step of each case comes from its device step counter.
// Several cases in one launch (serving): case k owns workgroups cases[k].wg0 .. + its T, counted
// from cases[0].wg0; the first step of each case comes from its device step counter.
template <typename TB, bool MIXED, bool WARM>
__global__ __launch_bounds__(kLThreads) void k_emt_level_multi(LevelDev Ld, const LevelCase* cases, int n_cases,
                                                              int n_steps)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char L8[];
    __shared__ LevelCase cs;
    __shared__ int64_t s0;
    const int gb = (int)blockIdx.x + cases[0].wg0;
    int k = 0;
    for (int q = 1; q < n_cases; ++q)
        if (gb >= cases[q].wg0) k = q;
    {
        const int* src = (const int*)&cases[k];
        int* dst = (int*)&cs;
        for (int i = threadIdx.x; i < (int)(sizeof(LevelCase) / sizeof(int)); i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s0 = *cs.E.step;
        cs.P.n_steps = n_steps;
    }
    __syncthreads();
    level_body<TB, MIXED, WARM>(Ld, cs.D, cs.E, cs.H, cs.M, cs.P, s0, gb - cs.wg0, L8);
}

template <typename TB, bool MIXED, bool WARM>
static hipError_t launch_level_t(const LevelDev& D, const EmtDev& E, const HierDev& H, const ModDev& M,
                                 const RunParams& P, hipStream_t s)
{
    const size_t lds = level_layout<TB, MIXED>(D, M.R).total;
    const void* fn = (const void*)k_emt_level<TB, MIXED, WARM>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0, per = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kLThreads, lds);
    if (e != hipSuccess) return e;
    if (per * cus < D.T) return hipErrorCooperativeLaunchTooLarge;
    LevelDev Dc = D;
    EmtDev Ec = E;
    HierDev Hc = H;
    ModDev Mc = M;
    RunParams Pc = P;
    void* args[] = {&Dc, &Ec, &Hc, &Mc, &Pc};
    e = hipMemsetAsync(D.sync, 0, (size_t)D.T * sizeof(unsigned int), s);
    if (e != hipSuccess) return e;
    e = hipLaunchCooperativeKernel(fn, dim3(D.T), dim3(kLThreads), args, (unsigned int)lds, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_emt_level(const LevelDev& D, const EmtDev& E, const HierDev& H, const ModDev& M, const RunParams& P,
                            int prec, hipStream_t s)
{
    if (prec == HINV_FP64)
        return P.warm ? launch_level_t<double, true, true>(D, E, H, M, P, s) : launch_level_t<double, false, false>(D, E, H, M, P, s);
    if (P.warm) return launch_level_t<float, true, true>(D, E, H, M, P, s);
    return launch_level_t<float, true, false>(D, E, H, M, P, s);
}

template <typename TB, bool MIXED, bool WARM>
static hipError_t launch_level_multi_t(const LevelDev& Ld, int R, const LevelCase* d_cases, const int* n_wg,
                                       unsigned int* const* sync, int n_cases, int n_steps, hipStream_t s)
{
    const size_t lds = level_layout<TB, MIXED>(Ld, R).total;
    const void* fn = (const void*)k_emt_level_multi<TB, MIXED, WARM>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0, per = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kLThreads, lds);
    if (e != hipSuccess) return e;
    const int cap = per * cus;
    // consecutive launches over runs of cases whose workgroups fit the GPU at once
    for (int k = 0; k < n_cases; ++k) {
        if (n_wg[k] > cap) return hipErrorCooperativeLaunchTooLarge;
        e = hipMemsetAsync(sync[k], 0, (size_t)n_wg[k] * sizeof(unsigned int), s);
        if (e != hipSuccess) return e;
    }
    int k = 0;
    while (k < n_cases) {
        int k1 = k, wgs = 0;
        while (k1 < n_cases && wgs + n_wg[k1] <= cap) wgs += n_wg[k1++];
        LevelDev Lc = Ld;
        const LevelCase* dc = d_cases + k;
        int nc = k1 - k, ns = n_steps;
        void* args[] = {&Lc, &dc, &nc, &ns};
        e = hipLaunchCooperativeKernel(fn, dim3(wgs), dim3(kLThreads), args, (unsigned int)lds, s);
        if (e != hipSuccess) return e;
        k = k1;
    }
    return hipGetLastError();
}

hipError_t launch_emt_level_multi(const LevelDev& Ld, int R, const LevelCase* d_cases, const int* n_wg,
                                  unsigned int* const* sync, int n_cases, int n_steps, int prec, int warm, hipStream_t s)
{
    if (prec == HINV_FP64)
        return warm ? launch_level_multi_t<double, true, true>(Ld, R, d_cases, n_wg, sync, n_cases, n_steps, s)
                    : launch_level_multi_t<double, false, false>(Ld, R, d_cases, n_wg, sync, n_cases, n_steps, s);
    if (warm) return launch_level_multi_t<float, true, true>(Ld, R, d_cases, n_wg, sync, n_cases, n_steps, s);
    return launch_level_multi_t<float, true, false>(Ld, R, d_cases, n_wg, sync, n_cases, n_steps, s);
}

}  // namespace hinv
