// Team stepping of one EMT case: one workgroup per leaf of the partition
// tree, all steps in one cooperative launch (paper Section II, Eq. (1)-(2);
// coupling levels as in Section III.B made exact; line changes as the SMW
// correction standing in for Section IV's update).
//
// Each workgroup holds in LDS: its leaf block B_l^{-1}, every capacitance
// inverse S_t^{-1}, the Z-panel rows of its own buses and of its "X rows"
// (coupling-column endpoints, tie-line neighbours, line-loss endpoints), the
// SMW vectors at those rows, and the case state of its buses.  Per apply:
//   1. own rows: v0 = B_l^{-1} x (LDS GEMV), published in a global exchange
//      vector (double-buffered by apply parity);
//   2. one team barrier;
//   3. every workgroup reads v0 at its X rows and computes, redundantly, every
//      level's y = S^{-1} U^T v (all levels in two phases: each column's s from
//      v0 and a precomputed row that folds in the lower levels' corrections of
//      the column's row, then y = S^{-1} s), then the corrected values of its
//      own rows and X rows, then the SMW correction.
// Rows shared by two workgroups are computed with identical operations in
// both, so their values agree bitwise and the history update of a tie line
// (and the refinement residual) needs no second exchange.  FP32 storage refines
// against the FP64 residual; FP64 storage warm-started runs the incremental form
// v = v_prev + P (b - G v_prev), one apply per step.
#include "hinv_internal.h"
#include "team_sync.h"

namespace hinv {

constexpr int kTeamThreads = 1024;
constexpr int kTeamWaves = kTeamThreads / 64;
constexpr int kGemvLanes = 8;           // leaf GEMV: lanes per row (column chunks), summed by DPP
constexpr int kSub = 4;                 // lanes per coupling-column sum s_g (quad sums)
constexpr int kSub8 = 8;                // lanes per y_g and per final-update row (sums over eight lanes)
static_assert(kMaxLeaf <= kTeamThreads, "one own row per thread in the right-hand side");
static_assert(kMaxLeaf * kGemvLanes <= kTeamThreads, "one row per group of GEMV lanes");

template <typename TB>
struct TAcc { using T = float; };
template <>
struct TAcc<double> { using T = double; };

struct TeamLayout {
    size_t blk, sall, zown, xz, uown, ux, acoef;
    size_t b, v, t, d, xv, xd, s, y, h0, h1, hC, gC, oval, bg, bal, samp, sph, sn, colw, cinv, mdg, red, tz;
    size_t xrow, xupd, utab, otab, xpos, cm, cc0, cso, ylist, lvlc, orp, ocol, bglob, bf, bt, iptr, ibr, sptr;
    size_t aoff, alo, alen;
    size_t lpa, lpb, loa, lob, mact, lbr, lst, vg, ctl;
    size_t total;
};

template <typename TB>
__host__ __device__ inline TeamLayout team_layout(const TeamDev& T, int R, bool refines)
{
    TeamLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = (o + bytes + 15) & ~(size_t)15;
        return r;
    };
    const size_t NL = T.NL, NX = T.NX, H = T.H, nc = T.nc;
    // FP32 storage refines against G in FP64, and so does the incremental FP64 form (its residual);
    // the direct FP64 path has no use for G's rows or the correction vectors, and its LDS is the
    // tighter one
    L.blk = take(sizeof(TB) * NL * NL);
    L.sall = take(sizeof(TB) * (size_t)T.sent);
    L.zown = take(sizeof(TB) * (size_t)T.ZO);
    L.xz = take(sizeof(TB) * (size_t)T.XZU);
    L.uown = take(sizeof(TB) * R * NL);
    L.ux = take(sizeof(TB) * R * NX);
    L.acoef = take(sizeof(TB) * (size_t)T.nA);
    const size_t D = sizeof(double);
    L.b = take(D * NL); L.v = take(D * NL);
    L.t = take(refines ? D * NL : 0); L.d = take(refines ? D * NL : 0);
    L.xv = take(D * NX); L.xd = take(refines ? D * NX : 0);
    L.s = take(D * nc); L.y = take(D * nc);
    L.h0 = take(D * T.NB); L.h1 = take(D * T.NB);
    L.hC = take(D * NL); L.gC = take(D * NL);
    L.oval = take(refines ? D * T.NE : 0); L.bg = take(D * T.NB); L.bal = take(D * T.NB);
    L.samp = take(D * T.NS); L.sph = take(D * T.NS); L.sn = take(D * T.NS);
    L.colw = take(D * nc);
    L.cinv = take(D * R * R * R); L.mdg = take(D * R);
    L.red = take(D * 2 * kTeamWaves); L.tz = take(D * 2 * R);
    const size_t I = sizeof(int);
    L.xrow = take(I * NX); L.xupd = take(I * NX);
    L.utab = take(sizeof(int4) * NX * H); L.otab = take(sizeof(int4) * H);
    L.xpos = take(I * nc); L.cm = take(I * nc); L.cc0 = take(I * nc); L.cso = take(I * nc);
    L.ylist = take(I * T.NY);
    L.lvlc = take(I * (H + 1));
    L.orp = take(refines ? I * (NL + 1) : 0); L.ocol = take(refines ? I * T.NE : 0);
    L.aoff = take(I * nc); L.alo = take(I * nc); L.alen = take(I * nc);
    L.bglob = take(I * T.NB); L.bf = take(I * T.NB); L.bt = take(I * T.NB);
    L.iptr = take(I * (NL + 1)); L.ibr = take(I * T.NI); L.sptr = take(I * (NL + 1));
    L.lpa = take(I * R); L.lpb = take(I * R); L.loa = take(I * R); L.lob = take(I * R);
    L.mact = take(I * R); L.lbr = take(I * R); L.lst = take(I * R);
    L.vg = take(sizeof(unsigned long long));
    L.ctl = take(I * 8);
    L.total = o;
    return L;
}

size_t team_lds_bytes(const TeamDev& T, const HierDev& H, int R, int prec, int warm)
{
    (void)H;
    return prec == HINV_FP64 ? team_layout<double>(T, R, warm != 0).total : team_layout<float>(T, R, true).total;
}

template <typename TB, bool MIXED, bool WARM>
__global__ __launch_bounds__(kTeamThreads) void k_emt_team(TeamDev T, EmtDev E, HierDev H, ModDev M, RunParams P)
{
    using TA = typename TAcc<TB>::T;
    // MIXED with FP64 storage is the incremental form v = v_prev + P (b - G v_prev): one FP64 apply of
    // the residual per step, no convergence statistics
    constexpr bool INC = MIXED && sizeof(TB) == 8;
    static_assert(MIXED || sizeof(TB) == 8, "FP32 storage refines");
    static_assert(!INC || WARM, "the incremental FP64 form starts from the previous step's voltages");
    extern __shared__ __attribute__((aligned(16))) unsigned char L8[];
    const int R = M.R;
    const TeamLayout Ly = team_layout<TB>(T, R, MIXED);
    const int w = blockIdx.x, tid = threadIdx.x;
    const int n = H.n, NL = T.NL, NX = T.NX, Hn = T.H, nc = T.nc;
    const int lo = T.w_lo[w], nl = T.w_nl[w], nx = T.w_nx[w], nb = T.w_nb[w], nxu = T.w_nxu[w], ny = T.w_ny[w];
    TB* blk = (TB*)(L8 + Ly.blk);
    TB* sall = (TB*)(L8 + Ly.sall);
    TB* zown = (TB*)(L8 + Ly.zown);
    TB* xz = (TB*)(L8 + Ly.xz);
    TB* uown = (TB*)(L8 + Ly.uown);
    TB* ux = (TB*)(L8 + Ly.ux);
    TB* acoef = (TB*)(L8 + Ly.acoef);
    double* b = (double*)(L8 + Ly.b);
    double* v = (double*)(L8 + Ly.v);
    double* t = (double*)(L8 + Ly.t);
    double* d = (double*)(L8 + Ly.d);
    double* xv = (double*)(L8 + Ly.xv);
    double* xd = (double*)(L8 + Ly.xd);
    double* s = (double*)(L8 + Ly.s);
    double* y = (double*)(L8 + Ly.y);
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
    double* colw = (double*)(L8 + Ly.colw);
    double* cinv = (double*)(L8 + Ly.cinv);
    double* mdg = (double*)(L8 + Ly.mdg);
    double* red = (double*)(L8 + Ly.red);
    double* tz = (double*)(L8 + Ly.tz);
    int* xrow = (int*)(L8 + Ly.xrow);
    int* xupd = (int*)(L8 + Ly.xupd);
    int4* utab = (int4*)(L8 + Ly.utab);   // per updated X row and level: Z offset (-1: none), columns,
                                          // first column, X position
    int4* otab = (int4*)(L8 + Ly.otab);   // the same for the own rows
    int* xpos = (int*)(L8 + Ly.xpos);
    int* cm = (int*)(L8 + Ly.cm);
    int* cc0 = (int*)(L8 + Ly.cc0);
    int* cso = (int*)(L8 + Ly.cso);
    int* ylist = (int*)(L8 + Ly.ylist);   // columns whose y this workgroup computes
    int* lvlc = (int*)(L8 + Ly.lvlc);
    int* orp = (int*)(L8 + Ly.orp);
    int* ocol = (int*)(L8 + Ly.ocol);
    int* bglob = (int*)(L8 + Ly.bglob);
    int* bf = (int*)(L8 + Ly.bf);
    int* bt = (int*)(L8 + Ly.bt);
    int* iptr = (int*)(L8 + Ly.iptr);
    int* ibr = (int*)(L8 + Ly.ibr);
    int* sptr = (int*)(L8 + Ly.sptr);
    int* aoff = (int*)(L8 + Ly.aoff);
    int* alo = (int*)(L8 + Ly.alo);
    int* alen = (int*)(L8 + Ly.alen);
    int* lpa = (int*)(L8 + Ly.lpa);
    int* lpb = (int*)(L8 + Ly.lpb);
    int* loa = (int*)(L8 + Ly.loa);
    int* lob = (int*)(L8 + Ly.lob);
    int* mact = (int*)(L8 + Ly.mact);
    int* lbr = (int*)(L8 + Ly.lbr);
    int* lst = (int*)(L8 + Ly.lst);
    unsigned long long* vg = (unsigned long long*)(L8 + Ly.vg);
    int* ctl = (int*)(L8 + Ly.ctl);

    const TB* gblk;
    const TB* gS;
    const TB* gZ;
    const TB* gU;
    const TB* gA;
    if constexpr (sizeof(TB) == 8) {
        gblk = (const TB*)H.blk; gS = (const TB*)H.Sinv; gZ = (const TB*)H.Z; gU = (const TB*)M.U;
        gA = (const TB*)T.acoef;
    } else {
        gblk = (const TB*)H.blk32; gS = (const TB*)H.Sinv32; gZ = (const TB*)H.Z32; gU = (const TB*)M.U32;
        gA = (const TB*)T.acoef32;
    }
    // ---------------- load the workgroup's tables and state into LDS
    {
        const TB* src = gblk + H.leaf_off[w];
        for (int i = tid; i < nl * nl; i += kTeamThreads) blk[i] = src[i];
        for (int k = tid; k < ny; k += kTeamThreads) {      // the needed rows of every S^{-1}
            const int g = T.ylist[(int64_t)w * nc + k];
            ylist[k] = g;
            const int node = H.col_node[g];
            const int m = H.node_m[node], q = g - H.node_col0[node], ld = T.cld[(int64_t)w * nc + g];
            const TB* src = gS + H.node_soff[node] + q;
            TB* dst = sall + T.csop[(int64_t)w * nc + g];
            for (int p = 0; p < m; ++p) dst[p * ld] = src[(int64_t)p * m];
        }
        const int* wxrow = T.xrow + (int64_t)w * NX;
        for (int x = tid; x < nx; x += kTeamThreads) xrow[x] = wxrow[x];
        for (int q = tid; q < T.w_nxu[w]; q += kTeamThreads) xupd[q] = T.xupd[(int64_t)w * NX + q];
        for (int i = tid; i < nxu * Hn; i += kTeamThreads) {     // updated X rows: tables and Z values
            const int q = i / Hn, h = i - q * Hn;
            const int x = T.xupd[(int64_t)w * NX + q];
            const int64_t gi = ((int64_t)w * NX + x) * Hn + h;
            const int zo = T.uzo[(int64_t)w * NX * Hn + i], pm = T.xpm[gi];
            utab[i] = make_int4(zo, pm, T.xpc[gi], x);
            if (zo >= 0) {
                const int P = T.xpan[gi];
                const TB* zp = gZ + H.pan_zoff[P] + (wxrow[x] - H.pan_lo[P]);
                for (int j = 0; j < pm; ++j) xz[zo + j] = zp[(int64_t)j * H.pan_n[P]];
            }
        }
        for (int h = 0; h < Hn; ++h) {
            const int zo = T.ozo[w * Hn + h];
            if (tid == 0) otab[h] = make_int4(zo, T.opm[w * Hn + h], T.opc[w * Hn + h], 0);
            if (zo >= 0) {
                const int P = T.opan[w * Hn + h], pm = T.opm[w * Hn + h];
                const TB* zp = gZ + H.pan_zoff[P] + (lo - H.pan_lo[P]);
                for (int i = tid; i < pm * nl; i += kTeamThreads) {
                    const int j = i / nl, r = i - j * nl;
                    zown[zo + i] = zp[(int64_t)j * H.pan_n[P] + r];
                }
            }
        }
        for (int g = tid; g < nc; g += kTeamThreads) {
            xpos[g] = T.xpos[(int64_t)w * nc + g];
            const int node = H.col_node[g];
            cm[g] = H.node_m[node] | (T.cld[(int64_t)w * nc + g] << 16);   // order | leading dimension << 16
            cc0[g] = H.node_col0[node];
            cso[g] = T.csop[(int64_t)w * nc + g];
            colw[g] = H.col_w[g];
            aoff[g] = T.aoff[g];
            alo[g] = T.alo[g];
            alen[g] = T.alen[g];
        }
        for (int i = tid; i < T.nA; i += kTeamThreads) acoef[i] = gA[i];
        for (int h = tid; h <= Hn; h += kTeamThreads) lvlc[h] = H.lvl_col[h];
        const int* worp = T.orp + (int64_t)w * (NL + 1);
        for (int r = tid; r <= nl; r += kTeamThreads) {
            if (MIXED) orp[r] = worp[r];
            iptr[r] = T.iptr[(int64_t)w * (NL + 1) + r];
            sptr[r] = T.sptr[(int64_t)w * (NL + 1) + r];
        }
        if (MIXED) {
            for (int e = tid; e < worp[nl]; e += kTeamThreads) {
                ocol[e] = T.ocol[(int64_t)w * T.NE + e];
                oval[e] = T.oval[(int64_t)w * T.NE + e];
            }
        }
        for (int q = tid; q < nb; q += kTeamThreads) {
            const int64_t gq = (int64_t)w * T.NB + q;
            bglob[q] = T.bglob[gq];
            bf[q] = T.bf[gq];
            bt[q] = T.bt[gq];
            bg[q] = T.bg[gq];
            bal[q] = T.bal[gq];
            hc[q] = E.h[(int64_t)(P.step0 & 1) * E.n_cases * E.nbr + T.bglob[gq]];
        }
        for (int i = tid; i < T.iptr[(int64_t)w * (NL + 1) + nl]; i += kTeamThreads) ibr[i] = T.ibr[(int64_t)w * T.NI + i];
        for (int i = tid; i < T.sptr[(int64_t)w * (NL + 1) + nl]; i += kTeamThreads) {
            samp[i] = T.samp[(int64_t)w * T.NS + i];
            sph[i] = T.sph[(int64_t)w * T.NS + i];
        }
        for (int r = tid; r < nl; r += kTeamThreads) {
            b[r] = E.b[lo + r];
            v[r] = E.v[lo + r];
            hC[r] = E.hC[lo + r];
            gC[r] = E.gC[lo + r];
        }
        for (int x = tid; x < nx; x += kTeamThreads) xv[x] = E.v[wxrow[x]];
        // line changes of the case (case 0): activation steps, endpoints as X / own indices
        const int cnt = R > 0 ? M.count[0] : 0;
        if (tid == 0) ctl[1] = cnt;
        if (tid < cnt) {
            mact[tid] = M.act[tid];
            mdg[tid] = M.dg[tid];
            const int a = M.a[tid], bb = M.b[tid];
            int pa = -1, pb = -1;
            for (int x = 0; x < nx; ++x) {
                if (wxrow[x] == a) pa = x;
                if (wxrow[x] == bb) pb = x;
            }
            lpa[tid] = pa;
            lpb[tid] = bb >= 0 ? pb : -1;
            loa[tid] = (a >= lo && a < lo + nl) ? a - lo : -1;
            lob[tid] = (bb >= lo && bb < lo + nl) ? bb - lo : -1;
            if (pa < 0 || (bb >= 0 && pb < 0)) atomicOr(P.flags, kFlagTeamRow);
        }
        for (int i = tid; i < R * R * R; i += kTeamThreads) cinv[i] = M.Cinv[i];
        for (int i = tid; i < cnt * nl; i += kTeamThreads) {
            const int j = i / nl, r = i - j * nl;
            uown[j * NL + r] = gU[(int64_t)j * n + lo + r];
        }
        for (int i = tid; i < cnt * nx; i += kTeamThreads) {
            const int j = i / nx, x = i - j * nx;
            ux[j * NX + x] = gU[(int64_t)j * n + wxrow[x]];
        }
        const int nlost = E.loss_cnt[0];
        if (tid == 0) ctl[2] = nlost;
        if (tid < nlost) {
            lbr[tid] = E.loss_br[tid];
            lst[tid] = E.loss_step[tid];
        }
    }
    __syncthreads();
    const int cnt = ctl[1], nlost = ctl[2];
    int par = 0;
    unsigned int epoch = 0;
    bool alive = true;
    double worst = 0.0;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform in the wavefront
    const int ns = sptr[nl];
    int64_t sn_step = -1;
    const int my_perm = tid < nl ? E.perm[lo + tid] : 0;   // caller's index of this thread's row (records)

    // one application of the stored inverse (with the active line changes):
    // out (own rows), outx (X rows) from xin (own rows)
    auto apply = [&](const double* xin, double* out, double* outx, int ract, bool want_vm) -> bool {
        // kGemvLanes lanes per row r = tid / kGemvLanes, lane c of the group takes the block columns
        // j = c (mod kGemvLanes); the group's partial sums are added by DPP moves (quads, then the
        // two quads of each half row), and the group's first lane stores the row
        double* X0 = T.X0 + (int64_t)par * n;
        {
            const int r = tid / kGemvLanes, c = tid % kGemvLanes;
            const bool act = r < nl;    // whole groups of kGemvLanes lanes are active or not
            TA acc = 0;
            if (act)
                for (int j = c; j < nl; j += kGemvLanes) acc += (TA)blk[j * nl + r] * (TA)xin[j];
            double val = quad_sum((double)acc);
            val += half_row_mirror(val);
            if (act && c == 0) {
                out[r] = val;
                xchg_store(&X0[lo + r], val);
            }
        }
        count_arrive(T.sync);
        ++epoch;
        if (sn_step >= 0) {      // source injections of the next step, by the last wavefront, while wavefront 0 polls
            if (tid >= kTeamThreads - 64)
                for (int q = tid - (kTeamThreads - 64); q < ns; q += 64)
                    sn[q] = samp[q] * sin(E.omega * ((double)sn_step * E.dt) + sph[q]);
            sn_step = -1;
        }
        if (!count_wait(T.sync, T.T, epoch, P.flags, ctl)) return false;
        if (want_vm) {   // the team's largest |v| (vg was cleared before the barrier)
            for (int i = tid; i < T.T; i += kTeamThreads)
                atomicMax(vg, (unsigned long long)__double_as_longlong(xchg_load(&T.VM[(int64_t)par * T.T + i])));
        }
        for (int x = tid; x < nx; x += kTeamThreads) outx[x] = xchg_load(&X0[xrow[x]]);
        __syncthreads();
        // coupling levels, all at once: s_g = w_g u_g - a_g . u from the leaf-apply values u at the
        // column rows (a_g carries the lower levels' corrections of the row), then y = S^{-1} s;
        // kSub lanes share each column's s (quad sums), kSub8 lanes each y (eight-lane sums); all rows
        // are updated at the end.
        if (nc > 0) {
            for (int idx = tid; idx < nc * kSub; idx += kTeamThreads) {
                const int g = idx / kSub, sub = idx & (kSub - 1);
                const int a0 = aoff[g], al = alo[g], an = alen[g];
                TA acc = 0;
                for (int k = sub; k < an; k += kSub) acc += (TA)acoef[a0 + k] * (TA)outx[xpos[al + k]];
                acc = quad_sum(acc);
                if (sub == 0) s[g] = colw[g] * outx[xpos[g]] - (double)acc;
            }
            __syncthreads();
            for (int idx = tid; idx < ny * kSub8; idx += kTeamThreads) {
                const int g = ylist[idx / kSub8], sub = idx & (kSub8 - 1);
                const int m = cm[g] & 0xffff, ld = cm[g] >> 16, q0 = cc0[g];
                const TB* Si = sall + cso[g];
                TA acc = 0;
                for (int p = sub; p < m; p += kSub8) acc += (TA)Si[p * ld] * (TA)s[q0 + p];
                acc = oct_sum(acc);
                if (sub == 0) y[g] = (double)acc;
            }
            __syncthreads();
        }
        // v -= sum over levels of Z y, on the X rows whose final values this workgroup uses (G
        // neighbours, line-loss endpoints: first nxu items) and the own rows, kSub8 lanes per row; every
        // level's table entry is loaded first, so that the levels' loads are in flight together.  The
        // other X rows (coupling-column rows only) keep v0: nothing reads them before the next exchange.
        for (int idx = tid; Hn > 0 && idx < (nxu + nl) * kSub8; idx += kTeamThreads) {
            const int i = idx / kSub8, sub = idx & (kSub8 - 1);
            const bool isx = i < nxu;
            const int r = i - nxu;
            int4 tb[kTeamMaxLevels];
#pragma unroll
            for (int h = 0; h < kTeamMaxLevels; ++h)
                if (h < Hn) tb[h] = isx ? utab[i * Hn + h] : otab[h];
            const int x = tb[0].w;
            TA acc[kTeamMaxLevels];
#pragma unroll
            for (int h = 0; h < kTeamMaxLevels; ++h) {
                acc[h] = 0;
                if (h < Hn && tb[h].x >= 0) {
                    const int zo = tb[h].x, pm = tb[h].y, pc = tb[h].z;
                    if (isx) {
                        for (int j = sub; j < pm; j += kSub8) acc[h] += (TA)xz[zo + j] * (TA)y[pc + j];
                    } else {
                        for (int j = sub; j < pm; j += kSub8) acc[h] += (TA)zown[zo + j * nl + r] * (TA)y[pc + j];
                    }
                }
            }
            double val = isx ? outx[x] : out[r];
#pragma unroll
            for (int h = 0; h < kTeamMaxLevels; ++h) {
                if (h < Hn) {
                    const TA a = oct_sum(acc[h]);
                    if (tb[h].x >= 0) val -= (double)a;
                }
            }
            if (sub == 0) {
                if (isx) outx[x] = val;
                else out[r] = val;
            }
        }
        __syncthreads();
        if (ract > 0) {
            if (tid < ract) tz[tid] = outx[lpa[tid]] - (lpb[tid] >= 0 ? outx[lpb[tid]] : 0.0);
            __syncthreads();
            if (tid < ract) {
                const double* Ci = cinv + (ract - 1) * R * R;
                double acc = 0.0;
                for (int j = 0; j < ract; ++j) acc += Ci[tid * R + j] * tz[j];
                tz[R + tid] = acc;
            }
            __syncthreads();
            for (int r = tid; r < nl; r += kTeamThreads) {
                double acc = 0.0;
                for (int j = 0; j < ract; ++j) acc += (double)uown[j * NL + r] * tz[R + j];
                out[r] -= acc;
            }
            for (int q = tid; q < nxu; q += kTeamThreads) {
                const int x = xupd[q];
                double acc = 0.0;
                for (int j = 0; j < ract; ++j) acc += (double)ux[j * NX + x] * tz[R + j];
                outx[x] -= acc;
            }
            __syncthreads();
        }
        par ^= 1;
        return true;
    };

    // t = b - G_step v on own rows (FP64), then v += P t
    auto refine = [&](int ract, bool last) -> bool {
        for (int r = tid; r < nl; r += kTeamThreads) {
            double acc = 0.0;
            for (int e = orp[r]; e < orp[r + 1]; ++e) {
                const int c = ocol[e];
                acc += oval[e] * (c < nl ? v[c] : xv[c - nl]);
            }
            for (int j = 0; j < ract; ++j) {
                if (loa[j] != r && lob[j] != r) continue;
                const double wv = xv[lpa[j]] - (lpb[j] >= 0 ? xv[lpb[j]] : 0.0);
                acc += (loa[j] == r ? 1.0 : -1.0) * mdg[j] * wv;
            }
            t[r] = b[r] - acc;
        }
        if (last) {        // publish this workgroup's max |v| for the team-wide norm
            double vm = 0.0;
            for (int r = tid; r < nl; r += kTeamThreads) vm = fmax(vm, fabs(v[r]));
            for (int o = 32; o > 0; o >>= 1) vm = fmax(vm, __shfl_xor(vm, o));
            if (lane == 0) red[kTeamWaves + wave] = vm;
            __syncthreads();
            if (tid == 0) {
                double V = 0.0;
                for (int q = 0; q < kTeamWaves; ++q) V = fmax(V, red[kTeamWaves + q]);
                xchg_store(&T.VM[(int64_t)par * T.T + w], V);
                *vg = 0ull;
            }
        }
        __syncthreads();
        if (!apply(t, d, xd, ract, last)) return false;
        double dm = 0.0;
        for (int r = tid; r < nl; r += kTeamThreads) {
            v[r] += d[r];
            dm = fmax(dm, fabs(d[r]));
        }
        for (int x = tid; x < nx; x += kTeamThreads) xv[x] += xd[x];
        if (last) {        // max |d| over the own rows / the team's max |v|
            for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o));
            if (lane == 0) red[wave] = dm;
            __syncthreads();
            if (tid == 0) {
                double D = 0.0;
                for (int q = 0; q < kTeamWaves; ++q) D = fmax(D, red[q]);
                const double V = __longlong_as_double((long long)*vg);
                const double ratio = V > 0.0 ? D / V : (D > 0.0 ? INFINITY : 0.0);
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
    for (int it = 0; it < P.n_steps && alive; ++it) {
        const int64_t step = P.step0 + it;
        sn_step = step + 1;      // the step's first apply computes the next step's source injections
        int ract = 0;
        while (ract < cnt && (int64_t)mact[ract] <= step) ++ract;
        if (!MIXED) {
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
        for (int q = tid; q < nb; q += kTeamThreads) {
            const int e = bglob[q];
            bool lost = false;
            for (int j = 0; j < nlost; ++j)
                if (lbr[j] == e && (int64_t)lst[j] <= step + 1) lost = true;
            double hv = 0.0;
            if (!lost) {
                const int f = bf[q], to = bt[q];
                const double vft = (f < nl ? v[f] : xv[f - nl]) - (to < nl ? v[to] : xv[to - nl]);
                const double ie = bg[q] * vft + hc[q];
                hv = bg[q] * vft + bal[q] * ie;
            }
            hn[q] = hv;
        }
        __syncthreads();
        const int64_t j = step - P.step0;
        if (tid < nl) {          // one own row per thread
            const int r = tid;
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
            const int64_t o = j * (int64_t)n + my_perm;
            if (P.v_rec) P.v_rec[o] = va;
            if (P.b_rec) P.b_rec[o] = b[r];
            b[r] = bn;
        }
        double* tmp = hc;
        hc = hn;
        hn = tmp;
        __syncthreads();
        if (P.clk && w == 0 && tid == 0 && j < P.clk_cap) P.clk[j] = (int64_t)wall_clock64();
    }
    if (!alive) return;
    const int64_t nstep = P.step0 + P.n_steps;
    for (int r = tid; r < nl; r += kTeamThreads) {
        E.b[lo + r] = b[r];
        E.v[lo + r] = v[r];
        E.hC[lo + r] = hC[r];
    }
    for (int q = tid; q < nb; q += kTeamThreads)
        if (T.bown[(int64_t)w * T.NB + q]) E.h[(int64_t)(nstep & 1) * E.n_cases * E.nbr + bglob[q]] = hc[q];
    if (tid == 0) {
        if (MIXED && !INC && P.stats) atomicMax(&P.stats[0], (unsigned long long)__double_as_longlong(worst));
        if (w == 0) {
            if (P.applies) atomicAdd(&P.applies[0], (unsigned long long)applies);
            *E.step = nstep;
        }
    }
}

template <typename TB, bool MIXED, bool WARM>
static hipError_t launch_team_t(const TeamDev& T, const EmtDev& E, const HierDev& H, const ModDev& M,
                                const RunParams& P, hipStream_t s)
{
    const size_t lds = team_layout<TB>(T, M.R, MIXED).total;
    const void* fn = (const void*)k_emt_team<TB, MIXED, WARM>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    TeamDev Tc = T;
    EmtDev Ec = E;
    HierDev Hc = H;
    ModDev Mc = M;
    RunParams Pc = P;
    void* args[] = {&Tc, &Ec, &Hc, &Mc, &Pc};
    e = hipMemsetAsync(T.sync, 0, (size_t)T.T * sizeof(unsigned int), s);
    if (e != hipSuccess) return e;
    e = hipLaunchCooperativeKernel(fn, dim3(T.T), dim3(kTeamThreads), args, (unsigned int)lds, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_emt_team(const TeamDev& T, const EmtDev& E, const HierDev& H, const ModDev& M, const RunParams& P,
                           int prec, hipStream_t s)
{
    if (prec == HINV_FP64)
        return P.warm ? launch_team_t<double, true, true>(T, E, H, M, P, s) : launch_team_t<double, false, false>(T, E, H, M, P, s);
    if (P.warm) return launch_team_t<float, true, true>(T, E, H, M, P, s);
    return launch_team_t<float, true, false>(T, E, H, M, P, s);
}

// ---------------- the rows a_g of the two-phase coupling levels
//
// Bottom-up over the levels, as maps from u (the leaf-apply values at the
// column rows), for the columns g of level h and every column c:
//   am[g][c] = w_g sum_{hh<h} sum_j Z_hh[row_g][p_j] bm[p_j][c]   (p_j: the
//              columns of the row's level-hh panel; zero on the lowest level),
//   bm[g][c] = sum_p S_t^{-1}[p][q_g] (w_{c0+p} [c = c0+p] - am[c0+p][c])
//              (t: the column's node, columns c0 .. c0+m-1, q_g = g - c0),
// so that s = diag(w) u - am u and y = bm u, as the sequential levels give.
struct CouplingMap {
    int nc, Hn;
    const int* cpan;
    double* am;
    double* bm;
};

__global__ void k_coupling_am(HierDev H, CouplingMap D, int h)
{
    const int nc = D.nc, g0 = H.lvl_col[h - 1];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)(H.lvl_col[h] - g0) * nc) return;
    const int g = g0 + (int)(i / nc), c = (int)(i % nc);
    const int r = H.col_row[g];
    double acc = 0.0;
    for (int hh = 1; hh < h; ++hh) {
        const int pp = D.cpan[(int64_t)g * D.Hn + hh - 1];
        if (pp < 0) continue;
        const double* zp = H.Z + H.pan_zoff[pp] + (r - H.pan_lo[pp]);
        const int p0 = H.pan_col0[pp], pn = H.pan_n[pp];
        for (int j = 0; j < H.pan_m[pp]; ++j) acc += zp[(int64_t)j * pn] * D.bm[(int64_t)(p0 + j) * nc + c];
    }
    D.am[(int64_t)g * nc + c] = H.col_w[g] * acc;
}

__global__ void k_coupling_bm(HierDev H, CouplingMap D, int h)
{
    const int nc = D.nc, g0 = H.lvl_col[h - 1];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)(H.lvl_col[h] - g0) * nc) return;
    const int g = g0 + (int)(i / nc), c = (int)(i % nc);
    const int t = H.col_node[g], m = H.node_m[t], c0 = H.node_col0[t];
    const double* Si = H.Sinv + H.node_soff[t] + (g - c0);
    double acc = 0.0;
    for (int p = 0; p < m; ++p) {
        const int gp = c0 + p;
        const double sv = (gp == c ? H.col_w[gp] : 0.0) - D.am[(int64_t)gp * nc + c];
        acc += Si[(int64_t)p * m] * sv;
    }
    D.bm[(int64_t)g * nc + c] = acc;
}

hipError_t launch_coupling_map(const HierDev& H, int Hn, int nc, const int* cpan, double* am, double* bm,
                               hipStream_t s)
{
    if (nc <= 0) return hipSuccess;
    std::vector<int> lvl(Hn + 1);
    hipError_t e = hipMemcpyAsync(lvl.data(), H.lvl_col, sizeof(int) * (Hn + 1), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const CouplingMap D{nc, Hn, cpan, am, bm};
    for (int h = 1; h <= Hn; ++h) {
        const int64_t cnt = (int64_t)(lvl[h] - lvl[h - 1]) * nc;
        if (cnt <= 0) continue;
        const int blocks = (int)((cnt + 255) / 256);
        k_coupling_am<<<blocks, 256, 0, s>>>(H, D, h);
        k_coupling_bm<<<blocks, 256, 0, s>>>(H, D, h);
    }
    return hipGetLastError();
}

__global__ void k_team_apack(TeamDev D)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= D.nc) return;
    const int a0 = D.aoff[g], al = D.alo[g];
    for (int k = 0; k < D.alen[g]; ++k) {
        const double a = D.am[(int64_t)g * D.nc + al + k];
        D.acoef[a0 + k] = a;
        D.acoef32[a0 + k] = (float)a;
    }
}

hipError_t launch_team_acoef(const TeamDev& T, const HierDev& H, hipStream_t s)
{
    if (T.nc <= 0) return hipSuccess;
    hipError_t e = launch_coupling_map(H, T.H, T.nc, T.cpan, T.am, T.bm, s);
    if (e != hipSuccess) return e;
    k_team_apack<<<(T.nc + 255) / 256, 256, 0, s>>>(T);
    return hipGetLastError();
}

}  // namespace hinv
