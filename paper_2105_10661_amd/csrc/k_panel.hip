// Panel stepping of EMT cases that share one base network: the batched form
// of the hierarchical apply.  Cases advance in panels of kPanelCases columns;
// a team of one workgroup per leaf of the partition tree owns one panel, and
// all steps run in one cooperative launch (paper Section II, Eq. (1)-(2);
// coupling levels of Section III.B made exact; line changes as per-case SMW
// corrections standing in for Section IV's update).
//
// Per apply, in every workgroup of a team:
//   1. own rows: V0 = B_l^{-1} X for the whole panel as one matrix product on
//      the matrix cores (16x16x4 MFMA; the leaf block stays in registers as A
//      fragments for the whole launch).  The values at the leaf's coupling-
//      column rows are published in the team's exchange (indexed by column,
//      double-buffered by apply parity), and so is the workgroup's share of
//      each case's w^T V0 = u^T X (u = G0^{-1} w, G0 symmetric) over its rows;
//   2. one team barrier;
//   3. u, the leaf-apply values at every column row, is read from the
//      exchange; the y of every column the workgroup applies is y = M u (M:
//      the coupling levels folded into one map) on the matrix cores; own rows
//      and X rows subtract their Z rows times y; then each case's SMW
//      correction with its w^T V0 summed over the team in workgroup order.
// Rows shared by two workgroups (a line between leaves) get identical
// operations in both: every y is formed by the same k-step groups wherever it
// is computed, and own rows and X rows use one dot-product order, so the
// history of a tie line, kept by the workgroups of both endpoints, stays
// bitwise consistent without a second exchange.
#include "hinv_internal.h"
#include "team_sync.h"

namespace hinv {

constexpr int kPThreads = 512;                 // 8 wavefronts: 2 per SIMD, up to 256 VGPRs each
constexpr int kPWaves = kPThreads / 64;
constexpr int kPB = kPanelCases;
constexpr int kPRowItems = (kPanelMaxLeaf * kPanelCases + kPThreads - 1) / kPThreads;   // (row, case) items
constexpr int kPUItems = (kPanelMaxCols * kPanelCases + kPThreads - 1) / kPThreads;     // (column, case) items
constexpr int kPXItems = (kPanelMaxX * kPanelCases + kPThreads - 1) / kPThreads;        // (X row, case) items
constexpr int kPMaxFrag = 18;     // A fragments per wavefront (leaf <= 96 rows, see panel_gemm)
constexpr int kPHelpTiles = 3;    // row tiles of each helper wavefront
constexpr int kPHelpK = 6;        // k-steps of a tile's tail
constexpr int kPYT = kPanelYTasksPerWave;
constexpr int kPHItems = 6;       // (branch, case) items of a thread in the history update (<= 192 branches)
// residual entries loaded ahead of their multiply-adds: 2 with FP64 storage, 3 with FP32 (measured; the
// FP64 form holds more registers across the residual, and larger batches there cost more than they hide)
template <typename TB> constexpr int kRW = sizeof(TB) == 8 ? 2 : 3;
static_assert(kPB == 16, "the panel is the N dimension of a 16x16x4 MFMA");
static_assert(kPThreads % kPB == 0, "all items of a thread belong to one case");
static_assert(kPWaves == kPanelWaves, "wavefront count shared with the host plan");

template <typename TB>
struct PAcc { using T = float; };
template <>
struct PAcc<double> { using T = double; };

typedef double pd4 __attribute__((ext_vector_type(4)));
typedef float pf4 __attribute__((ext_vector_type(4)));

// D(16x16) += A(16x4) B(4x16).  Lane l holds A[l%16][l/16] and B[l/16][l%16];
// element i of its accumulator is D[row(l, i)][l%16], where row differs
// between the FP64 and the FP32 instruction (measured on gfx950).
template <typename TB>
struct Mfma16;
template <>
struct Mfma16<double> {
    using V = pd4;
    __device__ static __forceinline__ V op(double a, double b, V c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
    // element and lane of D[r][c]
    __device__ static __forceinline__ int elem(int r) { return r >> 2; }
    __device__ static __forceinline__ int lane(int r, int c) { return ((r & 3) << 4) | c; }
};
template <>
struct Mfma16<float> {
    using V = pf4;
    __device__ static __forceinline__ V op(float a, float b, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
    __device__ static __forceinline__ int elem(int r) { return r & 3; }
    __device__ static __forceinline__ int lane(int r, int c) { return ((r >> 2) << 4) | c; }
};

__device__ __forceinline__ double pfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float pfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// sum_j z[j*zs] * y[(ps+j)*kPB + c] over the slots ps .. ps+pm-1, accumulated in TA (one helper for
// own rows and X rows keeps shared rows bitwise identical)
template <typename TA, typename TB>
__device__ __forceinline__ TA pdot(const TB* z, int zs, const double* y, int ps, int pm, int c)
{
    TA acc = 0;
    for (int j = 0; j < pm; ++j) acc = pfma((TA)z[j * zs], (TA)y[(ps + j) * kPB + c], acc);
    return acc;
}

// The same chain with the operands loaded eight at a time ahead of the multiply-adds (identical
// arithmetic, so rows computed by pdot and by pdot_pf agree bitwise).
template <typename TA, typename TB>
__device__ __forceinline__ TA pdot_pf(const TB* z, int zs, const double* y, int ps, int pm, int c)
{
    TA acc = 0;
    for (int j0 = 0; j0 < pm; j0 += 8) {
        TA zz[8], yy[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int j = j0 + k < pm ? j0 + k : pm - 1;
            zz[k] = (TA)z[j * zs];
            yy[k] = (TA)y[(ps + j) * kPB + c];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (j0 + k < pm) acc = pfma(zz[k], yy[k], acc);
    }
    return acc;
}

// Split of the leaf product (MT row tiles of 16, KS k-steps of 4): wavefront t < MT takes the first KM
// k-steps of tile t; the last KT = KS - KM k-steps of every tile go to the helper wavefronts 6 and 7
// (tile t to helper t % 2), whose results meet the main ones through LDS.  With MT = 6 every SIMD
// (wavefronts w and w + 4) issues the same number of products.
struct PanelGemm {
    int MT, KS, KM, KT;
};
__host__ __device__ inline PanelGemm panel_gemm(int NLp)
{
    PanelGemm g;
    g.MT = NLp / 16;
    g.KS = NLp / 4;
    const int h = (g.MT + 1) / 2;                    // tiles per helper
    g.KM = (g.KS * h + h) / (h + 1);                 // ceil(KS h / (h + 1))
    g.KT = g.KS - g.KM;
    return g;
}
static_assert(kPWaves == 8, "six main and two helper wavefronts");

struct PanelLayout {
    size_t stat;         // end of the per-leaf tables (the first bytes of the layout; copied from the leaf's image)
    size_t mfr, zown, xz, uo, ux;
    size_t b, v, td, xv, xd, U, yres, y, h, gC, oval, bg, bal, samp, sph, sn, cinv, mdg, tz, red, red2, red3;
    size_t xcol, xzo, xpm, xps, ozo, opm, ops, orp, ocol, iptr, ibr, sptr, prow, pubr, pubg, tk0, tnk, tfo, ttp,
        wtask, lpa, lpb, mact, cnt, ract, vg, ctl;
    size_t total;
};

// LDS layout.  FP64 (one apply per step) keeps b and v in one buffer: the
// leaf product overwrites b with v, and the right-hand side of the next step
// overwrites v row by row.  The incremental FP64 form (MIXED with FP64
// storage) forms its residual in place of b and keeps no convergence
// statistics.  The U region holds, in turn, the leaf product's partial sums,
// u (the exchanged values at the column rows) and the y tasks' results.
template <typename TB, bool MIXED>
__host__ __device__ inline PanelLayout panel_layout(const PanelDev& D, int R)
{
    constexpr bool INC = MIXED && sizeof(TB) == 8;
    PanelLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = (o + bytes + 15) & ~(size_t)15;
        return r;
    };
    const size_t NL = D.NL, NLp = D.NLp, NX = D.NX, NB = D.NB, H = D.H, B = kPB;
    const PanelGemm g = panel_gemm(D.NLp);
    size_t un = (size_t)D.ncp * B;
    if ((size_t)D.NT * 256 > un) un = (size_t)D.NT * 256;
    if ((size_t)g.MT * 256 > un) un = (size_t)g.MT * 256;
    const size_t S = sizeof(TB), F = sizeof(double), I = sizeof(int);
    // per-leaf tables (the same in every team; one image per leaf is copied at the launch)
    L.mfr = take(S * D.MF);
    L.zown = take(S * D.ZO);
    L.xz = take(S * D.XZ);
    L.gC = take(F * NL);
    L.oval = take(MIXED ? F * D.NE : 0);
    L.bg = take(F * NB);
    L.bal = take(F * NB);
    L.samp = take(F * D.NS);
    L.sph = take(F * D.NS);
    L.xcol = take(I * NX);
    L.xzo = take(I * NX * H);
    L.xpm = take(I * NX * H);
    L.xps = take(I * NX * H);
    L.ozo = take(I * H);
    L.opm = take(I * H);
    L.ops = take(I * H);
    L.orp = take(I * (NL + 1));
    L.ocol = take(MIXED ? I * D.NE : 0);
    L.iptr = take(I * (NL + 1));
    L.ibr = take(I * D.NI);
    L.sptr = take(I * (NL + 1));
    L.prow = take(I * NL);
    L.pubr = take(I * D.NP);
    L.pubg = take(I * D.NP);
    L.tk0 = take(I * D.NT);
    L.tnk = take(I * D.NT);
    L.tfo = take(I * D.NT);
    L.ttp = take(I * (D.NY / 16 + 1));
    L.wtask = take(I * kPWaves * kPYT);
    L.stat = o;
    // the team's cases and the state
    L.uo = take(S * R * NLp * B);
    L.ux = take(S * R * NX * B);
    L.b = take(F * NLp * B);
    L.v = MIXED ? take(F * NL * B) : L.b;
    L.td = INC ? L.b : take(MIXED ? F * NLp * B : 0);
    L.xv = take(F * NX * B);
    L.xd = take(MIXED ? F * NX * B : 0);
    L.U = take(F * un);
    L.yres = D.ysep ? take(F * D.NT * 256) : L.U;   // y task results (in the U region when LDS is short)
    L.y = take(F * D.NY * B);
    L.h = take(F * NB * B);
    L.sn = take(F * NL);          // source injection of each own row at the next step
    L.cinv = take(F * B * (R * (R + 1) * (2 * R + 1) / 6));   // per case the r x r inverses, r = 1..R, packed
    L.mdg = take(F * B * R);
    L.tz = take(F * B * 2 * R);
    L.red = take(MIXED && !INC ? F * 2 * kPWaves * B : 0);
    // red2 (shares per wavefront, before the barrier) and red3 (the team's shares, after it) share one region
    L.red2 = take(F * (kPWaves > D.T ? kPWaves : D.T) * R * B);
    L.red3 = L.red2;
    L.lpa = take(I * B * R);
    L.lpb = take(I * B * R);
    L.mact = take(I * B * R);
    L.cnt = take(I * B);
    L.ract = take(I * B);
    L.vg = take(sizeof(unsigned long long) * B);
    L.ctl = take(I * 8);
    L.total = o;
    return L;
}

size_t panel_lds_bytes(const PanelDev& D, int R, int prec, int warm)
{
    if (prec != HINV_FP64) return panel_layout<float, true>(D, R).total;
    return warm ? panel_layout<double, true>(D, R).total : panel_layout<double, false>(D, R).total;
}

// The per-leaf tables of the layout, written at base (LDS or a leaf's image in global memory) by nth
// threads: M fragments, Z rows of the own rows and X rows, y tasks, publish list, CSR rows, branch and
// source tables.
template <typename TB, bool MIXED>
__device__ void panel_fill_static(const PanelDev& D, const EmtDev& E, const HierDev& H, const PanelLayout& Ly,
                                  unsigned char* base, int l, int tid, int nth)
{
    const int Hn = D.H, NX = D.NX;
    const int lo = D.w_lo[l], nl = D.w_nl[l], nb = D.w_nb[l], nx = D.w_nx[l], ny = D.w_ny[l], nt = D.w_nt[l];
    const int npub = D.w_np[l];
    TB* mfr = (TB*)(base + Ly.mfr);
    TB* zown = (TB*)(base + Ly.zown);
    TB* xz = (TB*)(base + Ly.xz);
    double* gC = (double*)(base + Ly.gC);
    double* oval = (double*)(base + Ly.oval);
    double* bg = (double*)(base + Ly.bg);
    double* bal = (double*)(base + Ly.bal);
    double* samp = (double*)(base + Ly.samp);
    double* sph = (double*)(base + Ly.sph);
    int* xcol = (int*)(base + Ly.xcol);
    int* xzo = (int*)(base + Ly.xzo);
    int* xpm = (int*)(base + Ly.xpm);
    int* xps = (int*)(base + Ly.xps);
    int* ozo = (int*)(base + Ly.ozo);
    int* opm = (int*)(base + Ly.opm);
    int* ops = (int*)(base + Ly.ops);
    int* orp = (int*)(base + Ly.orp);
    int* ocol = (int*)(base + Ly.ocol);
    int* iptr = (int*)(base + Ly.iptr);
    int* ibr = (int*)(base + Ly.ibr);
    int* sptr = (int*)(base + Ly.sptr);
    int* prow = (int*)(base + Ly.prow);
    int* pubr = (int*)(base + Ly.pubr);
    int* pubg = (int*)(base + Ly.pubg);
    int* tk0 = (int*)(base + Ly.tk0);
    int* tnk = (int*)(base + Ly.tnk);
    int* tfo = (int*)(base + Ly.tfo);
    int* ttp = (int*)(base + Ly.ttp);
    int* wtask = (int*)(base + Ly.wtask);
    const TB* gZ;
    const TB* gM;
    if constexpr (sizeof(TB) == 8) {
        gZ = (const TB*)H.Z; gM = (const TB*)D.mfr;
    } else {
        gZ = (const TB*)H.Z32; gM = (const TB*)D.mfr32;
    }
    for (int i = tid; i < D.MF; i += nth) mfr[i] = gM[(int64_t)l * D.MF + i];
    for (int t = tid; t < nt; t += nth) {
        const int64_t gi = (int64_t)l * D.NT + t;
        tk0[t] = D.tk0[gi];
        tnk[t] = D.tnk[gi];
        tfo[t] = D.tfo[gi];
    }
    for (int t = tid; t <= ny / 16; t += nth) ttp[t] = D.ttp[(int64_t)l * (D.NY / 16 + 1) + t];
    for (int i = tid; i < kPWaves * kPYT; i += nth) wtask[i] = D.wtask[(int64_t)l * kPWaves * kPYT + i];
    const int64_t xb = (int64_t)l * NX;
    for (int x = tid; x < nx; x += nth) xcol[x] = D.xcol[xb + x];
    for (int i = tid; i < nx * Hn; i += nth) {
        const int64_t gi = xb * Hn + i;
        xzo[i] = D.xzo[gi];
        xpm[i] = D.xpm[gi];
        xps[i] = D.xps[gi];
    }
    for (int i = tid; i < D.w_xz[l]; i += nth) xz[i] = gZ[D.xzsrc[(int64_t)l * D.XZ + i]];
    for (int hh = tid; hh < Hn; hh += nth) {
        ozo[hh] = D.ozo[l * Hn + hh];
        opm[hh] = D.opm[l * Hn + hh];
        ops[hh] = D.ops[l * Hn + hh];
    }
    for (int hh = 0; hh < Hn; ++hh) {                    // own rows: Z panel rows at every level
        const int zo = D.ozo[l * Hn + hh];
        if (zo < 0) continue;
        const int pan = D.opan[l * Hn + hh], pm = D.opm[l * Hn + hh];
        const TB* zp = gZ + H.pan_zoff[pan] + (lo - H.pan_lo[pan]);
        for (int i = tid; i < pm * nl; i += nth) {
            const int j = i / nl, r = i - j * nl;
            zown[zo + i] = zp[(int64_t)j * H.pan_n[pan] + r];
        }
    }
    const int64_t rb = (int64_t)l * (D.NL + 1);
    for (int r = tid; r <= nl; r += nth) {
        orp[r] = D.orp[rb + r];
        iptr[r] = D.iptr[rb + r];
        sptr[r] = D.sptr[rb + r];
    }
    for (int q = tid; q < npub; q += nth) {
        pubr[q] = D.pubr[(int64_t)l * D.NP + q];
        pubg[q] = D.pubg[(int64_t)l * D.NP + q];
    }
    if (MIXED) {
        for (int e = tid; e < D.orp[rb + nl]; e += nth) {
            ocol[e] = D.ocol[(int64_t)l * D.NE + e];
            oval[e] = D.oval[(int64_t)l * D.NE + e];
        }
    }
    for (int i = tid; i < D.iptr[rb + nl]; i += nth) ibr[i] = D.ibr[(int64_t)l * D.NI + i];
    for (int i = tid; i < D.sptr[rb + nl]; i += nth) {
        samp[i] = D.samp[(int64_t)l * D.NS + i];
        sph[i] = D.sph[(int64_t)l * D.NS + i];
    }
    for (int q = tid; q < nb; q += nth) {
        const int64_t gq = (int64_t)l * D.NB + q;
        bg[q] = D.bg[gq];
        bal[q] = D.bal[gq];
    }
    for (int r = tid; r < nl; r += nth) {
        gC[r] = E.gC[lo + r];
        prow[r] = E.perm[lo + r];
    }
}

// MIXED with FP32 storage: FP64 refinement of the FP32 apply (warm: from the
// previous step's voltages).  MIXED with FP64 storage (INC): the incremental
// form v = v_prev + P (b - G v_prev), one FP64 apply per step.  In exact
// arithmetic it is P b; in floating point the apply's rounding scales with
// the change of v over a step rather than with v, which keeps the trajectory
// of a weakly damped mode (a bus left on its shunt capacitor alone by a line
// loss holds its voltage, an eigenvalue 1 of the step map) from drifting.
template <typename TB, bool MIXED, bool WARM>
__global__ __launch_bounds__(kPThreads) void k_emt_panel(PanelDev D, EmtDev E, HierDev H, ModDev M, RunParams P)
{
    using TA = typename PAcc<TB>::T;
    constexpr bool INC = MIXED && sizeof(TB) == 8;
    static_assert(!INC || WARM, "the incremental FP64 form starts from the previous step's voltages");
    extern __shared__ __attribute__((aligned(16))) unsigned char L8[];
    const int R = M.R;
    const PanelLayout Ly = panel_layout<TB, MIXED>(D, R);
    const int T = D.T, Hn = D.H, nc = D.nc, n = H.n, K = E.n_cases;
    const int l = blockIdx.x % T, team = D.team0 + blockIdx.x / T, tw = team * T + l;
    const int case0 = team * kPB;
    const int nvc = K - case0 < kPB ? K - case0 : kPB;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform in the wavefront
    const int lo = D.w_lo[l], nl = D.w_nl[l], nb = D.w_nb[l], nx = D.w_nx[l], ny = D.w_ny[l], nt = D.w_nt[l];
    const int npub = D.w_np[l];
    const int NLp = D.NLp, NX = D.NX, ncp = D.ncp;
    TB* mfr = (TB*)(L8 + Ly.mfr);
    TB* zown = (TB*)(L8 + Ly.zown);
    TB* xz = (TB*)(L8 + Ly.xz);
    TB* uo = (TB*)(L8 + Ly.uo);
    TB* ux = (TB*)(L8 + Ly.ux);
    double* b = (double*)(L8 + Ly.b);
    double* v = (double*)(L8 + Ly.v);
    double* td = (double*)(L8 + Ly.td);
    double* xv = (double*)(L8 + Ly.xv);
    double* xd = (double*)(L8 + Ly.xd);
    double* U = (double*)(L8 + Ly.U);
    double* yres = (double*)(L8 + Ly.yres);
    double* y = (double*)(L8 + Ly.y);
    double* h = (double*)(L8 + Ly.h);
    double* gC = (double*)(L8 + Ly.gC);
    double* oval = (double*)(L8 + Ly.oval);
    double* bg = (double*)(L8 + Ly.bg);
    double* bal = (double*)(L8 + Ly.bal);
    double* samp = (double*)(L8 + Ly.samp);
    double* sph = (double*)(L8 + Ly.sph);
    double* sn = (double*)(L8 + Ly.sn);
    double* cinv = (double*)(L8 + Ly.cinv);
    double* mdg = (double*)(L8 + Ly.mdg);
    double* tz = (double*)(L8 + Ly.tz);
    double* red = (double*)(L8 + Ly.red);
    double* red2 = (double*)(L8 + Ly.red2);
    int* xcol = (int*)(L8 + Ly.xcol);
    int* xzo = (int*)(L8 + Ly.xzo);
    int* xpm = (int*)(L8 + Ly.xpm);
    int* xps = (int*)(L8 + Ly.xps);
    int* ozo = (int*)(L8 + Ly.ozo);
    int* opm = (int*)(L8 + Ly.opm);
    int* ops = (int*)(L8 + Ly.ops);
    int* orp = (int*)(L8 + Ly.orp);
    int* ocol = (int*)(L8 + Ly.ocol);
    int* iptr = (int*)(L8 + Ly.iptr);
    int* ibr = (int*)(L8 + Ly.ibr);
    int* sptr = (int*)(L8 + Ly.sptr);
    int* prow = (int*)(L8 + Ly.prow);
    int* pubr = (int*)(L8 + Ly.pubr);
    int* pubg = (int*)(L8 + Ly.pubg);
    double* red3 = (double*)(L8 + Ly.red3);
    int* tk0 = (int*)(L8 + Ly.tk0);
    int* tnk = (int*)(L8 + Ly.tnk);
    int* tfo = (int*)(L8 + Ly.tfo);
    int* ttp = (int*)(L8 + Ly.ttp);
    int* wtask = (int*)(L8 + Ly.wtask);
    int* lpa = (int*)(L8 + Ly.lpa);
    int* lpb = (int*)(L8 + Ly.lpb);
    int* mact = (int*)(L8 + Ly.mact);
    int* cnt = (int*)(L8 + Ly.cnt);
    int* ract = (int*)(L8 + Ly.ract);
    unsigned long long* vg = (unsigned long long*)(L8 + Ly.vg);
    int* ctl = (int*)(L8 + Ly.ctl);

    const TB* gblk;
    const TB* gZ;
    const TB* gU;
    const TB* gM;
    if constexpr (sizeof(TB) == 8) {
        gblk = (const TB*)H.blk; gZ = (const TB*)H.Z; gU = (const TB*)M.U; gM = (const TB*)D.mfr;
    } else {
        gblk = (const TB*)H.blk32; gZ = (const TB*)H.Z32; gU = (const TB*)M.U32; gM = (const TB*)D.mfr32;
    }
    // ---------------- the leaf's tables (its image), the team's cases and the state, into LDS and
    // registers.  The global loads go in two rounds issued ahead of any use: first every value that needs
    // no other loaded value, then those addressed by the first round's indices; the LDS image is copied
    // while they are in flight.  (One loop per table costs a memory round trip each, ~18 us per launch.)
    // Every item of a thread belongs to case tid & 15 (512 threads, 16 cases).
    const int64_t xb = (int64_t)l * NX;
    const double* hsrc = E.h + (int64_t)(P.step0 & 1) * K * E.nbr;
    const int cme = tid & 15;
    const bool cok = cme < nvc;
    const int64_t crow = (int64_t)(case0 + cme) * n;        // the case's row block of n entries
    int gbr[kPHItems], hbft[kPHItems], hlost[kPHItems], xrw[kPXItems], rinc[kPRowItems];
    double lb[kPRowItems], lv[kPRowItems], hcr[kPRowItems];
    TB lu[kPanelMaxRank * kPRowItems];
    // round 1
    const int ucnt = cok ? M.count[case0 + cme] : 0;        // changes stored for the thread's case
#pragma unroll
    for (int k = 0; k < kPHItems; ++k) {
        const int i = tid + k * kPThreads, q = i >> 4;
        gbr[k] = q < nb ? D.bglob[(int64_t)l * D.NB + q] : 0;
        hbft[k] = q < nb ? D.hbft[(int64_t)l * D.NB + q] : 0;
        hlost[k] = q < nb ? D.hlost[(int64_t)tw * D.NB * kPB + i] : 0x7fffffff;
    }
#pragma unroll
    for (int k = 0; k < kPRowItems; ++k) {
        const int r = (tid + k * kPThreads) >> 4;
        const bool ok = r < nl && cok;
        lb[k] = ok ? E.b[crow + lo + r] : 0.0;
        lv[k] = (MIXED && ok) ? E.v[crow + lo + r] : 0.0;
        hcr[k] = ok ? E.hC[crow + lo + r] : 0.0;
        const int64_t rb = (int64_t)l * (D.NL + 1);
        rinc[k] = r < nl ? (D.iptr[rb + r] | ((D.iptr[rb + r + 1] - D.iptr[rb + r]) << 16)) : 0;
#pragma unroll
        for (int j = 0; j < kPanelMaxRank; ++j)      // u_j at own rows (any stored slot is a valid address)
            lu[j * kPRowItems + k] = (j < R && ok) ? gU[((int64_t)(case0 + cme) * R + j) * n + lo + r] : (TB)0;
    }
#pragma unroll
    for (int k = 0; k < kPXItems; ++k) {
        const int i = tid + k * kPThreads;
        xrw[k] = i < nx * kPB ? D.xrow[xb + (i >> 4)] : 0;
    }
    const TB* ablk = gblk + H.leaf_off[l];
    // round 2
    double lh[kPHItems], lx[kPXItems];
    TB lux[kPanelMaxRank * kPXItems];
#pragma unroll
    for (int k = 0; k < kPHItems; ++k) {
        const int q = (tid + k * kPThreads) >> 4;
        lh[k] = (q < nb && cok) ? hsrc[(int64_t)(case0 + cme) * E.nbr + gbr[k]] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kPXItems; ++k) {
        const bool ok = tid + k * kPThreads < nx * kPB && cok;
        lx[k] = ok ? E.v[crow + xrw[k]] : 0.0;
#pragma unroll
        for (int j = 0; j < kPanelMaxRank; ++j)
            lux[j * kPXItems + k] = (ok && j < R) ? gU[((int64_t)(case0 + cme) * R + j) * n + xrw[k]] : (TB)0;
    }
    // leaf block as A fragments (zero outside the leaf)
    const PanelGemm gm = panel_gemm(NLp);
    const bool mainw = wave < gm.MT, helper = wave >= 6;
    TB afrag[kPMaxFrag];          // zero outside the leaf and past the wavefront's k-steps
    {
#pragma unroll
        for (int f = 0; f < kPMaxFrag; ++f) {
            int t, ks;
            bool ok;
            if (helper) {
                t = (wave - 6) + 2 * (f / kPHelpK);
                ks = gm.KM + f % kPHelpK;
                ok = t < gm.MT && f % kPHelpK < gm.KT;
            } else {
                t = wave;
                ks = f;
                ok = mainw && f < gm.KM;
            }
            const int row = t * 16 + (lane & 15), col = ks * 4 + (lane >> 4);
            TB a = 0;
            if (ok && row < nl && col < nl) a = ablk[(int64_t)col * nl + row];
            afrag[f] = a;
        }
    }
    // the image copy while the loads above are in flight
    {
        const uint4* src = (const uint4*)(D.img + (int64_t)l * D.imgb);
        uint4* dst = (uint4*)L8;
        const int nq = (int)(Ly.stat / 16);
#pragma unroll 8
        for (int i = tid; i < nq; i += kPThreads) dst[i] = src[i];
    }
    if (tid < kPB) {                                    // line changes and losses of each case
        const int c = tid, k = case0 + c;
        const bool ok = c < nvc;
        cnt[c] = ok ? M.count[k] : 0;
        for (int j = 0; j < R; ++j) {
            mact[c * R + j] = ok ? M.act[k * R + j] : 0x7fffffff;
            mdg[c * R + j] = ok ? M.dg[k * R + j] : 0.0;
            lpa[c * R + j] = D.lpa[((int64_t)tw * kPB + c) * R + j];
            lpb[c * R + j] = D.lpb[((int64_t)tw * kPB + c) * R + j];
        }
        const int cs = R * (R + 1) * (2 * R + 1) / 6;
        for (int r = 1, o = 0; r <= R; o += r * r, ++r)
            for (int i = 0; i < r * r; ++i)
                cinv[c * cs + o + i] = ok ? M.Cinv[((int64_t)k * R + (r - 1)) * R * R + (i / r) * R + i % r] : 0.0;
        int ra = 0;                                     // changes active at the launch's first step
        while (ra < (ok ? M.count[k] : 0) && (int64_t)(ok ? M.act[k * R + ra] : 0x7fffffff) <= P.step0) ++ra;
        ract[c] = ra;
    }
    // the loaded values into LDS (rows beyond the leaf stay zero: product input)
#pragma unroll
    for (int k = 0; k < kPHItems; ++k) {
        const int i = tid + k * kPThreads;
        if ((i >> 4) < nb) h[i] = lh[k];
    }
#pragma unroll
    for (int k = 0; k < kPRowItems; ++k) {
        const int i = tid + k * kPThreads, r = i >> 4;
        if (i < NLp * kPB) {
            b[i] = lb[k];
            if (MIXED) {
                if (!INC) td[i] = 0.0;
                if (r < nl) v[i] = lv[k];
            }
#pragma unroll
            for (int j = 0; j < kPanelMaxRank; ++j)      // SMW vectors u_j at own rows ([j][r][c])
                if (j < R) uo[j * NLp * kPB + i] = j < ucnt ? lu[j * kPRowItems + k] : (TB)0;
        }
    }
#pragma unroll
    for (int k = 0; k < kPXItems; ++k) {
        const int i = tid + k * kPThreads;
        if (i < nx * kPB) xv[i] = lx[k];
#pragma unroll
        for (int j = 0; j < kPanelMaxRank; ++j)          // and at X rows ([j][x][c]), zero past nx
            if (j < R && i < NX * kPB) ux[j * NX * kPB + i] = (i < nx * kPB && j < ucnt) ? lux[j * kPXItems + k] : (TB)0;
    }
    __syncthreads();

    int par = 0;
    unsigned int epoch = D.epoch0;
    bool alive = true;
    double worst = 0.0;
    unsigned int* tflags = D.sync + (int64_t)team * T;
    int64_t sn_step = -1;    // the step whose source injections the next apply computes (-1: none)

    // value of a combined row index (own row or X row) in the pair (own, X)
    auto cval = [&](const double* own, const double* xr, int comb, int c) -> double {
        return comb < nl ? own[comb * kPB + c] : xr[(comb - nl) * kPB + c];
    };

    // one application of the stored inverse with each case's active changes:
    // out (own rows), outx (X rows) from xin (own rows, zero beyond nl); out
    // may be xin (it is written after every wavefront has read xin).  The
    // incremental FP64 form adds the result to v and xv instead of storing it
    // (out and outx then only hold intermediate values).
    auto apply = [&](const double* xin, double* out, double* outx, bool anyact, bool want_vm) -> bool {
        double* X0p = D.X0 + ((int64_t)team * 2 + par) * (int64_t)nc * kPB;
        double* SPp = D.SP + ((int64_t)team * 2 + par) * (int64_t)T * R * kPB;
        const double* VMp = D.VM + ((int64_t)team * 2 + par) * T * kPB;
        if (anyact) {   // this workgroup's share of u_j^T x per case (the thread's items all belong to case tid & 15)
            double sj[kPanelMaxRank];
#pragma unroll
            for (int j = 0; j < kPanelMaxRank; ++j) sj[j] = 0.0;
#pragma unroll
            for (int k = 0; k < kPRowItems; ++k) {
                const int i = tid + k * kPThreads;
                if (i < nl * kPB)
#pragma unroll
                    for (int j = 0; j < kPanelMaxRank; ++j)
                        if (j < R) sj[j] = pfma((double)uo[j * NLp * kPB + i], xin[i], sj[j]);
            }
#pragma unroll
            for (int j = 0; j < kPanelMaxRank; ++j) {
                sj[j] += __shfl_xor(sj[j], 16);
                sj[j] += __shfl_xor(sj[j], 32);
                if (j < R && lane < kPB) red2[(wave * R + j) * kPB + lane] = sj[j];
            }
        }
        {
            // rows past a wavefront's k-steps are clamped (their A fragments are zero)
            typename Mfma16<TB>::V acc = {0, 0, 0, 0};
            if (helper) {
#pragma unroll
                for (int i = 0; i < kPHelpTiles; ++i) {
                    typename Mfma16<TB>::V ht = {0, 0, 0, 0};
                    TB bop[kPHelpK];
#pragma unroll
                    for (int f = 0; f < kPHelpK; ++f) {
                        const int k = (gm.KM + f) * 4 + (lane >> 4);
                        bop[f] = (TB)xin[(k < NLp ? k : NLp - 1) * kPB + (lane & 15)];
                    }
#pragma unroll
                    for (int f = 0; f < kPHelpK; ++f) ht = Mfma16<TB>::op(afrag[i * kPHelpK + f], bop[f], ht);
                    const int t = (wave - 6) + 2 * i;
                    if (t < gm.MT)
#pragma unroll
                        for (int e = 0; e < 4; ++e) U[t * 256 + e * 64 + lane] = (double)ht[e];
                }
            } else if (mainw) {
#pragma unroll
                for (int f0 = 0; f0 < kPMaxFrag; f0 += kPHelpK) {
                    TB bop[kPHelpK];
#pragma unroll
                    for (int f = 0; f < kPHelpK; ++f) {
                        const int k = (f0 + f) * 4 + (lane >> 4);
                        bop[f] = (TB)xin[(k < NLp ? k : NLp - 1) * kPB + (lane & 15)];
                    }
#pragma unroll
                    for (int f = 0; f < kPHelpK; ++f) acc = Mfma16<TB>::op(afrag[f0 + f], bop[f], acc);
                }
            }
            __syncthreads();
            if (mainw) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const double val = (double)acc[i] + U[wave * 256 + i * 64 + lane];
                    const int r = wave * 16 + Mfma16<TB>::row(lane, i), c = lane & 15;
                    if (r < nl) out[r * kPB + c] = val;
                }
            }
            __syncthreads();
            // publish the values at the leaf's coupling-column rows, and the share of u^T x
            for (int i = tid; i < npub * kPB; i += kPThreads) {
                const int q = i >> 4, c = i & 15;
                xchg_store(&X0p[pubg[q] * kPB + c], out[pubr[q] * kPB + c]);
            }
            if (anyact && tid < R * kPB) {
                const int j = tid >> 4, c = tid & 15;
                double sw[kPWaves];
#pragma unroll
                for (int w = 0; w < kPWaves; ++w) sw[w] = red2[(w * R + j) * kPB + c];
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < kPWaves; ++w) s += sw[w];
                xchg_store(&SPp[((int64_t)l * R + j) * kPB + c], s);
            }
        }
        team_arrive(tflags, l, ++epoch);
        if (sn_step >= 0) {      // source injections of the next step, by the last wave, while wavefront 0 polls
            if (tid >= kPThreads - 64)
                for (int r = tid - (kPThreads - 64); r < nl; r += 64) {
                    double sr = 0.0;
                    for (int q = sptr[r]; q < sptr[r + 1]; ++q) sr += samp[q] * sin(E.omega * ((double)sn_step * E.dt) + sph[q]);
                    sn[r] = sr;
                }
            sn_step = -1;
        }
        if (!team_wait(tflags, T, epoch, P.flags, ctl)) return false;
        if (want_vm) {   // the team's largest |v| per case (vg was cleared before the barrier)
            for (int i = tid; i < T * kPB; i += kPThreads)
                atomicMax(&vg[i & 15], (unsigned long long)__double_as_longlong(xchg_load(&VMp[i])));
        }
        {   // every load of the exchange is issued before the first wait
            double ul[kPUItems], xl[kPXItems];
#pragma unroll
            for (int it = 0; it < kPUItems; ++it) {
                const int i = tid + it * kPThreads;
                ul[it] = i < nc * kPB ? xchg_load(&X0p[i]) : 0.0;
            }
#pragma unroll
            for (int it = 0; it < kPXItems; ++it) {
                const int i = tid + it * kPThreads;
                xl[it] = i < nx * kPB ? xchg_load(&X0p[xcol[i >> 4] * kPB + (i & 15)]) : 0.0;
            }
            const double spv = (anyact && tid < T * R * kPB) ? xchg_load(&SPp[tid]) : 0.0;   // the team's shares
            if (anyact && tid < T * R * kPB) red3[tid] = spv;
#pragma unroll
            for (int it = 0; it < kPUItems; ++it) {
                const int i = tid + it * kPThreads;
                if (i < ncp * kPB) U[i] = ul[it];
            }
#pragma unroll
            for (int it = 0; it < kPXItems; ++it) {
                const int i = tid + it * kPThreads;
                if (i < nx * kPB) outx[i] = xl[it];
            }
        }
        __syncthreads();
        if (anyact && tid < kPB) {   // w^T v0 of each active change (the shares in workgroup order), z = C^{-1} t
            const int c = tid, ra = ract[c];
            double t[kPanelMaxRank];
#pragma unroll
            for (int j = 0; j < kPanelMaxRank; ++j) {
                t[j] = 0.0;
                if (j < R)
                    for (int q0 = 0; q0 < T; q0 += 8) {
                        double v8[8];
#pragma unroll
                        for (int k = 0; k < 8; ++k) v8[k] = q0 + k < T ? red3[((q0 + k) * R + j) * kPB + c] : 0.0;
#pragma unroll
                        for (int k = 0; k < 8; ++k) t[j] += v8[k];
                    }
            }
            if (ra > 0) {
                const double* Ci = cinv + c * (R * (R + 1) * (2 * R + 1) / 6) + (ra - 1) * ra * (2 * ra - 1) / 6;
                for (int j = 0; j < ra; ++j) {
                    double z = 0.0;
                    for (int q = 0; q < ra; ++q) z += Ci[j * ra + q] * t[q];
                    tz[c * 2 * R + R + j] = z;
                }
            }
        }
        if (nc == 0) __syncthreads();        // z visible to the final update (no y phase in between)
        if (nc > 0) {
            // y = M u for the workgroup's slots: each task is one MFMA chain over an absolute group of
            // k-steps of one 16-row tile; a tile's tasks are summed in k order
            typename Mfma16<TB>::V yacc[kPYT];
#pragma unroll
            for (int k2 = 0; k2 < kPYT; ++k2) {
                yacc[k2] = typename Mfma16<TB>::V{0, 0, 0, 0};
                const int tk = __builtin_amdgcn_readfirstlane(wtask[wave * kPYT + k2]);
                if (tk >= 0) {
                    const int k0 = __builtin_amdgcn_readfirstlane(tk0[tk]);
                    const int nk = __builtin_amdgcn_readfirstlane(tnk[tk]);
                    const int fo = __builtin_amdgcn_readfirstlane(tfo[tk]);
                    for (int kk = 0; kk < nk; ++kk)
                        yacc[k2] = Mfma16<TB>::op(mfr[fo + kk * 64 + lane], (TB)U[(k0 + kk) * 64 + lane], yacc[k2]);
                }
            }
            if (!D.ysep) __syncthreads();     // the results overwrite u: every task has read it
#pragma unroll
            for (int k2 = 0; k2 < kPYT; ++k2) {
                const int tk = __builtin_amdgcn_readfirstlane(wtask[wave * kPYT + k2]);
                if (tk >= 0)
#pragma unroll
                    for (int e = 0; e < 4; ++e) yres[tk * 256 + e * 64 + lane] = (double)yacc[k2][e];
            }
            __syncthreads();
            for (int i = tid; i < ny * kPB; i += kPThreads) {     // a tile's tasks are consecutive, in k order
                const int s = i >> 4, c = i & 15, t = s >> 4, rr = s & 15;
                const int e = Mfma16<TB>::elem(rr), ln = Mfma16<TB>::lane(rr, c);
                double acc = 0.0;
                for (int q = ttp[t]; q < ttp[t + 1]; ++q) acc += yres[q * 256 + e * 64 + ln];
                y[i] = acc;
            }
            __syncthreads();
        }
        // own rows and X rows: v -= sum over levels of Z y (one dot-product order for every row, so
        // rows shared by two workgroups stay bitwise identical)
        if constexpr (sizeof(TB) == 8) {
            // own rows on the matrix cores, one 16-row tile per wavefront: the FP64 16x16x4 product
            // rounds as a chain of fused multiply-adds over k (measured bitwise on gfx950), which is
            // the chain the X-row loop below uses for the same rows in other workgroups
            if (mainw) {
                const int r0 = wave * 16, c = lane & 15;
                double val[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = r0 + Mfma16<TB>::row(lane, e);
                    val[e] = r < nl ? out[r * kPB + c] : 0.0;
                }
                const int ra_ = r0 + (lane & 15), rc = ra_ < nl ? ra_ : nl - 1;
                for (int hh = 0; hh < Hn; ++hh) {
                    const int zo = __builtin_amdgcn_readfirstlane(ozo[hh]);
                    if (zo < 0) continue;
                    const int pm = __builtin_amdgcn_readfirstlane(opm[hh]), ps = ops[hh];
                    typename Mfma16<TB>::V acc = {0, 0, 0, 0};
                    for (int k0 = 0; k0 < pm; k0 += 4) {
                        const int j = k0 + (lane >> 4), jc = j < pm ? j : pm - 1;
                        const TB a0 = zown[zo + jc * nl + rc];
                        const TB b0 = (TB)y[(ps + jc) * kPB + c];
                        acc = Mfma16<TB>::op((ra_ < nl && j < pm) ? a0 : (TB)0, j < pm ? b0 : (TB)0, acc);
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) val[e] -= (double)acc[e];
                }
                const int ra = anyact ? ract[c] : 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = r0 + Mfma16<TB>::row(lane, e);
                    double sa = 0.0;          // per-case SMW correction
                    for (int j = 0; j < ra; ++j)
                        sa = pfma((double)uo[j * NLp * kPB + r * kPB + c], tz[c * 2 * R + R + j], sa);
                    if (r < nl) {
                        if constexpr (INC) v[r * kPB + c] += val[e] - sa;
                        else out[r * kPB + c] = val[e] - sa;
                    }
                }
            }
        } else {
            for (int i = tid; i < nl * kPB; i += kPThreads) {
                const int r = i >> 4, c = i & 15;
                double val = out[i];
                for (int hh = 0; hh < Hn; ++hh) {
                    const int zo = ozo[hh];
                    if (zo >= 0) val -= (double)pdot<TA>(zown + zo + r, nl, y, ops[hh], opm[hh], c);
                }
                const int ra = anyact ? ract[c] : 0;
                double sa = 0.0;              // per-case SMW correction
                for (int j = 0; j < ra; ++j) sa = pfma((double)uo[j * NLp * kPB + i], tz[c * 2 * R + R + j], sa);
                if constexpr (INC) v[i] += val - sa;
                else out[i] = val - sa;
            }
        }
        // X rows, starting on the helper wavefronts (no own-row tile in the update above)
        for (int i = (tid + kPThreads - 6 * 64) % kPThreads; i < nx * kPB; i += kPThreads) {
            const int x = i >> 4, c = i & 15;
            double val = outx[i];
            for (int hh = 0; hh < Hn; ++hh) {
                const int zo = xzo[x * Hn + hh];
                if (zo >= 0) val -= (double)pdot_pf<TA>(xz + zo, 1, y, xps[x * Hn + hh], xpm[x * Hn + hh], c);
            }
            const int ra = anyact ? ract[c] : 0;
            double sa = 0.0;                  // per-case SMW correction
            for (int j = 0; j < ra; ++j) sa = pfma((double)ux[j * NX * kPB + i], tz[c * 2 * R + R + j], sa);
            if constexpr (INC) xv[i] += val - sa;
            else outx[i] = val - sa;
        }
        __syncthreads();
        par ^= 1;
        return true;
    };

    // t = b - G_step v on own rows (FP64), then v += P t; stats on the last pass.  The residual runs one
    // thread per (row, four cases): the row's CSR entries are loaded once for its four cases, whose
    // voltages sit next to each other (two 16-byte loads per entry); per case the entries are summed
    // in CSR order, then the case's active changes
    auto refine = [&](bool anyact, bool last) -> bool {
        for (int q = tid; q < nl * (kPB / 4); q += kPThreads) {
            const int r = q >> 2, c0 = (q & 3) * 4;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            const int e0 = orp[r], e1 = orp[r + 1];
            for (int eb = e0; eb < e1; eb += kRW<TB>) {
                double2 x[kRW<TB>][2];
                double w[kRW<TB>];
#pragma unroll
                for (int k = 0; k < kRW<TB>; ++k) {
                    const int e = eb + k < e1 ? eb + k : e1 - 1;
                    const int col = ocol[e];
                    w[k] = oval[e];
                    const double2* src = (const double2*)(col < nl ? v + col * kPB + c0 : xv + (col - nl) * kPB + c0);
                    x[k][0] = src[0];
                    x[k][1] = src[1];
                }
#pragma unroll
                for (int k = 0; k < kRW<TB>; ++k)
                    if (eb + k < e1) {
                        acc[0] += w[k] * x[k][0].x;
                        acc[1] += w[k] * x[k][0].y;
                        acc[2] += w[k] * x[k][1].x;
                        acc[3] += w[k] * x[k][1].y;
                    }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = c0 + u, ra = ract[c];
                for (int j = 0; j < ra; ++j) {
                    const int a = lpa[c * R + j], bb = lpb[c * R + j];
                    if (a != r && bb != r) continue;
                    const double wv = cval(v, xv, a, c) - (bb >= 0 ? cval(v, xv, bb, c) : 0.0);
                    acc[u] += (a == r ? 1.0 : -1.0) * mdg[c * R + j] * wv;
                }
            }
            const double2* bs = (const double2*)(b + r * kPB + c0);
            const double2 b0 = bs[0], b1 = bs[1];
            double2* ts = (double2*)(td + r * kPB + c0);
            ts[0] = double2{b0.x - acc[0], b0.y - acc[1]};
            ts[1] = double2{b1.x - acc[2], b1.y - acc[3]};
        }
        if (last) {        // publish this workgroup's max |v| per case for the team-wide norm
            double vm = 0.0;     // the thread's items all belong to case tid & 15
            for (int i = tid; i < nl * kPB; i += kPThreads) vm = fmax(vm, fabs(v[i]));
            vm = fmax(vm, __shfl_xor(vm, 16));
            vm = fmax(vm, __shfl_xor(vm, 32));
            if (lane < kPB) red[(kPWaves + wave) * kPB + lane] = vm;
            __syncthreads();
            if (tid < kPB) {
                double Vm = 0.0;
                for (int q = 0; q < kPWaves; ++q) Vm = fmax(Vm, red[(kPWaves + q) * kPB + tid]);
                xchg_store(&D.VM[(((int64_t)team * 2 + par) * T + l) * kPB + tid], Vm);
                vg[tid] = 0ull;
            }
        }
        __syncthreads();
        if (!apply(td, td, xd, anyact, last)) return false;
        if constexpr (INC) return true;          // the apply added its result to v and xv
        double dm = 0.0;     // the thread's items all belong to case tid & 15
        for (int i = tid; i < nl * kPB; i += kPThreads) {
            v[i] += td[i];
            dm = fmax(dm, fabs(td[i]));
        }
        for (int i = tid; i < nx * kPB; i += kPThreads) xv[i] += xd[i];
        if (last) {        // per case: max |d| over the own rows / the team's max |v|
            dm = fmax(dm, __shfl_xor(dm, 16));
            dm = fmax(dm, __shfl_xor(dm, 32));
            if (lane < kPB) red[wave * kPB + lane] = dm;
            __syncthreads();
            if (tid < nvc) {
                double Dm = 0.0;
                for (int q = 0; q < kPWaves; ++q) Dm = fmax(Dm, red[q * kPB + tid]);
                const double Vm = __longlong_as_double((long long)vg[tid]);
                const double ratio = Vm > 0.0 ? Dm / Vm : (Dm > 0.0 ? INFINITY : 0.0);
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
        const int64_t jr = step - P.rec_step0;
        const bool rec = jr >= 0 && jr < P.rec_cap;
        if ((!MIXED || INC) && rec && P.b_rec) {        // b is overwritten by v (the residual) below
            for (int i = tid; i < nl * kPB; i += kPThreads) {
                const int c = i & 15;
                if (c < nvc) P.b_rec[(jr * K + case0 + c) * (int64_t)n + prow[i >> 4]] = b[i];
            }
            __syncthreads();     // every thread has read b before the incremental form's residual replaces it
        }
        bool anyact = false;      // ract holds this step's active changes (set before the last barrier)
        for (int c = 0; c < kPB; ++c) anyact |= ract[c] > 0;
        if constexpr (!MIXED) {
            alive = apply(b, v, xv, anyact, false);
            applies += 1;
        } else {
            const int nref = INC ? 1 : (WARM ? P.max_refine + 1 : P.max_refine);
            if (!WARM) {
                alive = apply(b, v, xv, anyact, false);
                applies += 1;
            }
            for (int q = 0; q < nref && alive; ++q) {
                alive = refine(anyact, !INC && q == nref - 1);
                applies += 1;
            }
        }
        if (!alive) break;
        // history: new branch histories, then the right-hand side of step+1
#pragma unroll
        for (int k = 0; k < kPHItems; ++k) {
            const int i = tid + k * kPThreads, q = i >> 4, c = i & 15;
            if (q < nb) {
                const bool lost = (int64_t)hlost[k] <= step + 1;
                const double vft = cval(v, xv, hbft[k] & 0xffff, c) - cval(v, xv, hbft[k] >> 16, c);
                const double ie = bg[q] * vft + h[i];
                h[i] = lost ? 0.0 : bg[q] * vft + bal[q] * ie;
            }
        }
        __syncthreads();
        if (tid < kPB) {          // the next step's active changes (nothing reads ract until then)
            int ra = 0;
            while (ra < cnt[tid] && (int64_t)mact[tid * R + ra] <= step + 1) ++ra;
            ract[tid] = ra;
        }
#pragma unroll
        for (int k = 0; k < kPRowItems; ++k) {
            const int i = tid + k * kPThreads, r = i >> 4, c = i & 15;
            if (r < nl) {
                const double va = v[i];
                double bn = sn[r];
                const int q0 = rinc[k] & 0xffff, qn = rinc[k] >> 16;
                for (int qb = q0; qb < q0 + qn; qb += 4) {      // indices first, then the histories
                    int lb[4];
                    double hv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) lb[u] = ibr[qb + u < q0 + qn ? qb + u : q0 + qn - 1];
#pragma unroll
                    for (int u = 0; u < 4; ++u) hv[u] = h[(lb[u] >= 0 ? lb[u] : ~lb[u]) * kPB + c];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (qb + u < q0 + qn) bn -= lb[u] >= 0 ? hv[u] : -hv[u];
                }
                const double ic = gC[r] * va + hcr[k];
                const double hcn = -gC[r] * va - ic;
                hcr[k] = hcn;
                bn -= hcn;
                if (rec && c < nvc) {
                    const int64_t o = (jr * K + case0 + c) * (int64_t)n + prow[r];
                    if (P.v_rec) P.v_rec[o] = va;
                    if (MIXED && !INC && P.b_rec) P.b_rec[o] = b[i];
                }
                b[i] = bn;
            }
        }
        __syncthreads();
        if (P.clk && blockIdx.x == 0 && tid == 0 && step - P.step0 < P.clk_cap)
            P.clk[step - P.step0] = (int64_t)wall_clock64();
    }
    if (!alive) return;
    const int64_t nstep = P.step0 + P.n_steps;
    // FP64 keeps no v past the right-hand side: store b only (v is rebuilt by the next apply)
    for (int i = tid; i < nl * kPB; i += kPThreads) {
        const int r = i >> 4, c = i & 15;
        if (c < nvc) {
            const int64_t gi = (int64_t)(case0 + c) * n + lo + r;
            E.b[gi] = b[i];
            if (MIXED) E.v[gi] = v[i];
        }
    }
#pragma unroll
    for (int k = 0; k < kPRowItems; ++k) {
        const int i = tid + k * kPThreads, r = i >> 4, c = i & 15;
        if (r < nl && c < nvc) E.hC[(int64_t)(case0 + c) * n + lo + r] = hcr[k];
    }
    double* hdst = E.h + (int64_t)(nstep & 1) * K * E.nbr;
    for (int i = tid; i < nb * kPB; i += kPThreads) {
        const int q = i >> 4, c = i & 15;
        if (c < nvc && D.bown[(int64_t)l * D.NB + q]) hdst[(int64_t)(case0 + c) * E.nbr + D.bglob[(int64_t)l * D.NB + q]] = h[i];
    }
    if (tid < nvc) {
        if (MIXED && P.stats) atomicMax(&P.stats[case0 + tid], (unsigned long long)__double_as_longlong(worst));
        if (l == 0 && P.applies) atomicAdd(&P.applies[case0 + tid], (unsigned long long)applies);
    }
    if (blockIdx.x == 0 && tid == 0) *E.step = nstep;
}

// ---------------- M as the y tasks' A fragments: lane l of k-step kk of task t holds M[g][4 k + l/16] of
// the slot 16 tile + l%16 (g its column; zero for padding slots and columns beyond nc).  Grid (T, NT).
__global__ void k_panel_mfrag(PanelDev D)
{
    const int l = blockIdx.x, t = blockIdx.y;
    if (t >= D.w_nt[l]) return;
    const int64_t ti = (int64_t)l * D.NT + t;
    const int k0 = D.tk0[ti], nk = D.tnk[ti], fo = D.tfo[ti], tile = D.ttile[ti];
    double* m64 = const_cast<double*>(D.mfr) + (int64_t)l * D.MF + fo;
    float* m32 = const_cast<float*>(D.mfr32) + (int64_t)l * D.MF + fo;
    for (int i = threadIdx.x; i < nk * 64; i += blockDim.x) {
        const int kk = i >> 6, ln = i & 63;
        const int g = D.yslot[(int64_t)l * D.NY + tile * 16 + (ln & 15)];
        const int col = (k0 + kk) * 4 + (ln >> 4);
        const double val = (g >= 0 && col < D.nc) ? D.bm[(int64_t)g * D.nc + col] : 0.0;
        m64[i] = val;
        m32[i] = (float)val;
    }
}

hipError_t launch_panel_mfrag(const PanelDev& D, hipStream_t s)
{
    if (D.nc <= 0 || D.NT <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_panel_mfrag, dim3(D.T, D.NT), dim3(256), 0, s, D);
    return hipGetLastError();
}

// Each leaf's image of its tables (block l; the layout of the context's precision path).
template <typename TB, bool MIXED>
__global__ void k_panel_image(PanelDev D, EmtDev E, HierDev H, int R)
{
    const PanelLayout Ly = panel_layout<TB, MIXED>(D, R);
    panel_fill_static<TB, MIXED>(D, E, H, Ly, D.img + (int64_t)blockIdx.x * D.imgb, blockIdx.x, threadIdx.x, blockDim.x);
}

size_t panel_image_bytes(const PanelDev& D, int R, int prec, int warm)
{
    const size_t b = prec != HINV_FP64 ? panel_layout<float, true>(D, R).stat
                     : warm ? panel_layout<double, true>(D, R).stat : panel_layout<double, false>(D, R).stat;
    return (b + 255) / 256 * 256;
}

hipError_t launch_panel_image(const PanelDev& D, const EmtDev& E, const HierDev& H, int R, int prec, int warm,
                              hipStream_t s)
{
    if (prec != HINV_FP64) hipLaunchKernelGGL((k_panel_image<float, true>), dim3(D.T), dim3(256), 0, s, D, E, H, R);
    else if (warm) hipLaunchKernelGGL((k_panel_image<double, true>), dim3(D.T), dim3(256), 0, s, D, E, H, R);
    else hipLaunchKernelGGL((k_panel_image<double, false>), dim3(D.T), dim3(256), 0, s, D, E, H, R);
    return hipGetLastError();
}

template <typename TB, bool MIXED, bool WARM>
static const void* panel_fn()
{
    return (const void*)k_emt_panel<TB, MIXED, WARM>;
}

static const void* panel_kernel(int prec, int warm)
{
    if (prec == HINV_FP64) return warm ? panel_fn<double, true, true>() : panel_fn<double, false, false>();
    return warm ? panel_fn<float, true, true>() : panel_fn<float, true, false>();
}

hipError_t panel_setup(PanelDev& D, int R, int prec, int warm)
{
    const size_t lds = panel_lds_bytes(D, R, prec, warm);
    const void* fn = panel_kernel(prec, warm);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0, per = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kPThreads, lds);
    if (e != hipSuccess) return e;
    D.teams_per_launch = (per * cus) / D.T;     // teams that are co-resident in one launch
    if (D.teams_per_launch < 1) return hipErrorCooperativeLaunchTooLarge;
    return hipSuccess;
}

hipError_t launch_emt_panel(const PanelDev& D, const EmtDev& E, const HierDev& H, const ModDev& M, const RunParams& P,
                            int prec, hipStream_t s)
{
    const size_t lds = panel_lds_bytes(D, M.R, prec, P.warm);
    const void* fn = panel_kernel(prec, P.warm);
    if (D.teams_per_launch < 1) return hipErrorCooperativeLaunchTooLarge;
    for (int t0 = 0; t0 < D.n_teams; t0 += D.teams_per_launch) {
        const int nt = D.n_teams - t0 < D.teams_per_launch ? D.n_teams - t0 : D.teams_per_launch;
        PanelDev Dc = D;
        Dc.team0 = t0;
        EmtDev Ec = E;
        HierDev Hc = H;
        ModDev Mc = M;
        RunParams Pc = P;
        void* args[] = {&Dc, &Ec, &Hc, &Mc, &Pc};
        hipError_t e = hipLaunchCooperativeKernel(fn, dim3(nt * D.T), dim3(kPThreads), args, (unsigned int)lds, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace hinv
