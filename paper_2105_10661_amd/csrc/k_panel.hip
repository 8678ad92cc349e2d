// Panel stepping of EMT cases that share one base network: the batched form
// of the hierarchical apply.  Cases advance in panels of kPanelCases columns;
// a team of one workgroup per leaf of the partition tree owns one panel, and
// all steps run in one cooperative launch (paper Section II, Eq. (1)-(2);
// coupling levels of Section III.B made exact; line changes as per-case SMW
// corrections standing in for Section IV's update).
//
// Per apply, in every workgroup of a team:
//   1. own rows: V0 = B_l^{-1} X for the whole panel as one matrix product on
//      the matrix cores (16x16x4 MFMA; the leaf block B_l^{-1} stays in
//      registers as A fragments for the whole launch), published in the
//      team's exchange buffer (double-buffered by apply parity);
//   2. one team barrier;
//   3. the values at the coupling-column rows and at the X rows are read from
//      the exchange; every level's Y = S^{-1} U^T V is computed in every
//      workgroup, bottom-up, a column row's lower-level corrections applied
//      inline; own rows and X rows are corrected once at the end, then each
//      case's SMW correction follows.
// A row shared by two workgroups gets identical operations in both (one dot
// helper, the same operand order), so the history of a tie line, kept by the
// workgroups of both endpoints, stays bitwise consistent without a second
// exchange.
#include "hinv_internal.h"
#include "team_sync.h"

namespace hinv {

constexpr int kPThreads = 768;                 // 12 wavefronts: 3 per SIMD, ~168 VGPRs each
constexpr int kPWaves = kPThreads / 64;
constexpr int kPB = kPanelCases;
constexpr int kPRowItems = (kPanelMaxLeaf * kPanelCases + kPThreads - 1) / kPThreads;   // (row, case) items
constexpr int kPColItems = (kPanelMaxCols * kPanelCases + kPThreads - 1) / kPThreads;   // (column, case) items
constexpr int kPXItems = (kPanelMaxX * kPanelCases + kPThreads - 1) / kPThreads;        // (X row, case) items
constexpr int kPMaxFrag = 12;     // A fragments per wavefront (leaf <= 96 rows, see panel_gemm)
constexpr int kPLevelTiles = 2;   // 16-row tiles of the level solve per wavefront
static_assert(kPB == 16, "the panel is the N dimension of a 16x16x4 MFMA");
static_assert(kPThreads % kPB == 0, "all items of a thread belong to one case");

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
};
template <>
struct Mfma16<float> {
    using V = pf4;
    __device__ static __forceinline__ V op(float a, float b, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

__device__ __forceinline__ double pfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float pfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// sum_j z[j*zs] * y[(pc+j)*kPB + c], accumulated in TA (one helper for own
// rows, X rows and column rows keeps shared rows bitwise identical)
template <typename TA, typename TB>
__device__ __forceinline__ TA pdot(const TB* z, int zs, const double* y, int pc, int pm, int c)
{
    TA acc = 0;
    for (int j = 0; j < pm; ++j) acc = pfma((TA)z[j * zs], (TA)y[(pc + j) * kPB + c], acc);
    return acc;
}

// Split of the leaf product over the wavefronts: MT row tiles of 16, KS
// k-steps of 4; KSPLIT wavefronts share a row tile (partial sums through LDS).
struct PanelGemm {
    int MT, KS, KSPLIT, KSC;
};
__host__ __device__ inline PanelGemm panel_gemm(int NLp)
{
    PanelGemm g;
    g.MT = NLp / 16;
    g.KS = NLp / 4;
    const int a = kPWaves / g.MT, b = 1 + 8 / g.MT;
    g.KSPLIT = a < b ? a : b;
    g.KSC = (g.KS + g.KSPLIT - 1) / g.KSPLIT;
    return g;
}

struct PanelLayout {
    size_t sall, zown, xz, cz, uo, ux;
    size_t b, v, td, xv, xd, y, h, gC, colw, oval, bg, bal, samp, sph, sn, cinv, mdg, tz, red;
    size_t xrow, xzo, xpm, xpc, ozo, opm, opc, czo, cpm, cpc, crow, cm, cc0, cso, lvlc, orp, ocol, bglob, bf, bt, iptr,
        ibr, sptr, prow, lpa, lpb, mact, lbr, lst, cnt, nlost, ract, vg, ctl;
    size_t total;
};

// LDS layout.  FP64 (one apply per step) keeps b and v in one buffer: the
// leaf product overwrites b with v, and the right-hand side of the next step
// overwrites v row by row.  The y region also holds, in turn, the leaf
// product's partial sums, the raw values at the coupling-column rows and s.
template <typename TB, bool MIXED>
__host__ __device__ inline PanelLayout panel_layout(const PanelDev& D, int R)
{
    PanelLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = (o + bytes + 15) & ~(size_t)15;
        return r;
    };
    const size_t NL = D.NL, NLp = D.NLp, NX = D.NX, NB = D.NB, nc = D.nc, H = D.H, B = kPB;
    const PanelGemm g = panel_gemm(D.NLp);
    const size_t part = (size_t)(g.KSPLIT - 1) * g.MT * 256;
    const size_t yn = nc * B > part ? nc * B : part;
    const size_t S = sizeof(TB), F = sizeof(double), I = sizeof(int);
    L.sall = take(S * D.sent);
    L.zown = take(S * D.ZO);
    L.xz = take(S * D.XZ);
    L.cz = take(S * D.CZ);
    L.uo = take(S * R * NLp * B);
    L.ux = take(S * R * NX * B);
    L.b = take(F * NLp * B);
    L.v = MIXED ? take(F * NL * B) : L.b;
    L.td = take(MIXED ? F * NLp * B : 0);
    L.xv = take(F * NX * B);
    L.xd = take(MIXED ? F * NX * B : 0);
    L.y = take(F * yn);
    L.h = take(F * NB * B);
    L.gC = take(F * NL);
    L.colw = take(F * nc);
    L.oval = take(MIXED ? F * D.NE : 0);
    L.bg = take(F * NB);
    L.bal = take(F * NB);
    L.samp = take(F * D.NS);
    L.sph = take(F * D.NS);
    L.sn = take(F * D.NS);
    L.cinv = take(F * B * R * R * R);
    L.mdg = take(F * B * R);
    L.tz = take(F * B * 2 * R);
    L.red = take(MIXED ? F * 2 * kPWaves * B : 0);
    L.xrow = take(I * NX);
    L.xzo = take(I * NX * H);
    L.xpm = take(I * NX * H);
    L.xpc = take(I * NX * H);
    L.ozo = take(I * H);
    L.opm = take(I * H);
    L.opc = take(I * H);
    L.czo = take(I * nc * H);
    L.cpm = take(I * nc * H);
    L.cpc = take(I * nc * H);
    L.crow = take(I * nc);
    L.cm = take(I * nc);
    L.cc0 = take(I * nc);
    L.cso = take(I * nc);
    L.lvlc = take(I * (H + 1));
    L.orp = take(I * (NL + 1));
    L.ocol = take(MIXED ? I * D.NE : 0);
    L.bglob = take(I * NB);
    L.bf = take(I * NB);
    L.bt = take(I * NB);
    L.iptr = take(I * (NL + 1));
    L.ibr = take(I * D.NI);
    L.sptr = take(I * (NL + 1));
    L.prow = take(I * NL);
    L.lpa = take(I * B * R);
    L.lpb = take(I * B * R);
    L.mact = take(I * B * R);
    L.lbr = take(I * B * R);
    L.lst = take(I * B * R);
    L.cnt = take(I * B);
    L.nlost = take(I * B);
    L.ract = take(I * B);
    L.vg = take(sizeof(unsigned long long) * B);
    L.ctl = take(I * 8);
    L.total = o;
    return L;
}

size_t panel_lds_bytes(const PanelDev& D, int R, int prec)
{
    return prec == HINV_FP64 ? panel_layout<double, false>(D, R).total : panel_layout<float, true>(D, R).total;
}

template <typename TB, bool MIXED, bool WARM>
__global__ __launch_bounds__(kPThreads) void k_emt_panel(PanelDev D, EmtDev E, HierDev H, ModDev M, RunParams P)
{
    using TA = typename PAcc<TB>::T;
    extern __shared__ __attribute__((aligned(16))) unsigned char L8[];
    const int R = M.R;
    const PanelLayout Ly = panel_layout<TB, MIXED>(D, R);
    const int T = D.T, Hn = D.H, nc = D.nc, n = H.n, K = E.n_cases;
    const int l = blockIdx.x % T, team = D.team0 + blockIdx.x / T, tw = team * T + l;
    const int case0 = team * kPB;
    const int nvc = K - case0 < kPB ? K - case0 : kPB;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform in the wavefront
    const int lo = D.w_lo[l], nl = D.w_nl[l], nb = D.w_nb[l], nx = D.w_nx[tw];
    const int NLp = D.NLp;
    TB* sall = (TB*)(L8 + Ly.sall);
    TB* zown = (TB*)(L8 + Ly.zown);
    TB* xz = (TB*)(L8 + Ly.xz);
    TB* cz = (TB*)(L8 + Ly.cz);
    TB* uo = (TB*)(L8 + Ly.uo);
    TB* ux = (TB*)(L8 + Ly.ux);
    double* b = (double*)(L8 + Ly.b);
    double* v = (double*)(L8 + Ly.v);
    double* td = (double*)(L8 + Ly.td);
    double* xv = (double*)(L8 + Ly.xv);
    double* xd = (double*)(L8 + Ly.xd);
    double* y = (double*)(L8 + Ly.y);
    double* h = (double*)(L8 + Ly.h);
    double* gC = (double*)(L8 + Ly.gC);
    double* colw = (double*)(L8 + Ly.colw);
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
    int* xrow = (int*)(L8 + Ly.xrow);
    int* xzo = (int*)(L8 + Ly.xzo);
    int* xpm = (int*)(L8 + Ly.xpm);
    int* xpc = (int*)(L8 + Ly.xpc);
    int* ozo = (int*)(L8 + Ly.ozo);
    int* opm = (int*)(L8 + Ly.opm);
    int* opc = (int*)(L8 + Ly.opc);
    int* czo = (int*)(L8 + Ly.czo);
    int* cpm = (int*)(L8 + Ly.cpm);
    int* cpc = (int*)(L8 + Ly.cpc);
    int* crow = (int*)(L8 + Ly.crow);
    int* cm = (int*)(L8 + Ly.cm);
    int* cc0 = (int*)(L8 + Ly.cc0);
    int* cso = (int*)(L8 + Ly.cso);
    int* lvlc = (int*)(L8 + Ly.lvlc);
    int* orp = (int*)(L8 + Ly.orp);
    int* ocol = (int*)(L8 + Ly.ocol);
    int* bglob = (int*)(L8 + Ly.bglob);
    int* bf = (int*)(L8 + Ly.bf);
    int* bt = (int*)(L8 + Ly.bt);
    int* iptr = (int*)(L8 + Ly.iptr);
    int* ibr = (int*)(L8 + Ly.ibr);
    int* sptr = (int*)(L8 + Ly.sptr);
    int* prow = (int*)(L8 + Ly.prow);
    int* lpa = (int*)(L8 + Ly.lpa);
    int* lpb = (int*)(L8 + Ly.lpb);
    int* mact = (int*)(L8 + Ly.mact);
    int* lbr = (int*)(L8 + Ly.lbr);
    int* lst = (int*)(L8 + Ly.lst);
    int* cnt = (int*)(L8 + Ly.cnt);
    int* nlost = (int*)(L8 + Ly.nlost);
    int* ract = (int*)(L8 + Ly.ract);
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
    for (int g = tid; g < nc; g += kPThreads) {          // S^{-1} rows padded to m+1
        const int node = H.col_node[g];
        const int m = H.node_m[node], q = g - H.node_col0[node];
        const TB* src = gS + H.node_soff[node] + q;
        TB* dst = sall + D.csop[g];
        for (int p = 0; p < m; ++p) dst[p * (m + 1)] = src[(int64_t)p * m];
        crow[g] = H.col_row[g];
        cm[g] = m;
        cc0[g] = H.node_col0[node];
        cso[g] = D.csop[g];
        colw[g] = H.col_w[g];
    }
    for (int i = tid; i < nc * Hn; i += kPThreads) {     // column rows: Z values below the column's level
        const int zo = D.czo[i];
        czo[i] = zo;
        cpm[i] = D.cpm[i];
        cpc[i] = D.cpc[i];
        if (zo >= 0) {
            const int pan = D.cpan[i];
            const TB* zp = gZ + H.pan_zoff[pan] + (H.col_row[i / Hn] - H.pan_lo[pan]);
            for (int j = 0; j < D.cpm[i]; ++j) cz[zo + j] = zp[(int64_t)j * H.pan_n[pan]];
        }
    }
    const int64_t xb = (int64_t)tw * D.NX;
    for (int x = tid; x < nx; x += kPThreads) xrow[x] = D.xrow[xb + x];
    for (int i = tid; i < nx * Hn; i += kPThreads) {     // X rows: Z values at every level
        const int64_t gi = xb * Hn + i;
        const int zo = D.xzo[gi];
        xzo[i] = zo;
        xpm[i] = D.xpm[gi];
        xpc[i] = D.xpc[gi];
        if (zo >= 0) {
            const int pan = D.xpan[gi];
            const TB* zp = gZ + H.pan_zoff[pan] + (D.xrow[xb + i / Hn] - H.pan_lo[pan]);
            for (int j = 0; j < D.xpm[gi]; ++j) xz[zo + j] = zp[(int64_t)j * H.pan_n[pan]];
        }
    }
    for (int hh = 0; hh < Hn; ++hh) {                    // own rows: Z panel rows at every level
        const int zo = D.ozo[l * Hn + hh];
        if (tid == 0) { ozo[hh] = zo; opm[hh] = D.opm[l * Hn + hh]; opc[hh] = D.opc[l * Hn + hh]; }
        if (zo >= 0) {
            const int pan = D.opan[l * Hn + hh], pm = D.opm[l * Hn + hh];
            const TB* zp = gZ + H.pan_zoff[pan] + (lo - H.pan_lo[pan]);
            for (int i = tid; i < pm * nl; i += kPThreads) {
                const int j = i / nl, r = i - j * nl;
                zown[zo + i] = zp[(int64_t)j * H.pan_n[pan] + r];
            }
        }
    }
    for (int hh = tid; hh <= Hn; hh += kPThreads) lvlc[hh] = H.lvl_col[hh];
    {
        const int64_t rb = (int64_t)l * (D.NL + 1);
        for (int r = tid; r <= nl; r += kPThreads) {
            orp[r] = D.orp[rb + r];
            iptr[r] = D.iptr[rb + r];
            sptr[r] = D.sptr[rb + r];
        }
        if (MIXED) {
            for (int e = tid; e < D.orp[rb + nl]; e += kPThreads) {
                ocol[e] = D.ocol[(int64_t)l * D.NE + e];
                oval[e] = D.oval[(int64_t)l * D.NE + e];
            }
        }
        for (int i = tid; i < D.iptr[rb + nl]; i += kPThreads) ibr[i] = D.ibr[(int64_t)l * D.NI + i];
        for (int i = tid; i < D.sptr[rb + nl]; i += kPThreads) {
            samp[i] = D.samp[(int64_t)l * D.NS + i];
            sph[i] = D.sph[(int64_t)l * D.NS + i];
        }
    }
    for (int q = tid; q < nb; q += kPThreads) {
        const int64_t gq = (int64_t)l * D.NB + q;
        bglob[q] = D.bglob[gq];
        bf[q] = D.bf[gq];
        bt[q] = D.bt[gq];
        bg[q] = D.bg[gq];
        bal[q] = D.bal[gq];
    }
    for (int r = tid; r < nl; r += kPThreads) {
        gC[r] = E.gC[lo + r];
        prow[r] = E.perm[lo + r];
    }
    const double* hsrc = E.h + (int64_t)(P.step0 & 1) * K * E.nbr;
    for (int i = tid; i < nb * kPB; i += kPThreads) {
        const int q = i >> 4, c = i & 15;
        h[i] = c < nvc ? hsrc[(int64_t)(case0 + c) * E.nbr + D.bglob[(int64_t)l * D.NB + q]] : 0.0;
    }
    for (int i = tid; i < NLp * kPB; i += kPThreads) {  // rows beyond the leaf stay zero (product input)
        const int r = i >> 4, c = i & 15;
        const bool ok = r < nl && c < nvc;
        const int64_t gi = (int64_t)(case0 + c) * n + lo + r;
        b[i] = ok ? E.b[gi] : 0.0;
        if (MIXED) {
            td[i] = 0.0;
            if (r < nl) v[i] = ok ? E.v[gi] : 0.0;
        }
    }
    for (int i = tid; i < nx * kPB; i += kPThreads) {
        const int x = i >> 4, c = i & 15;
        xv[i] = c < nvc ? E.v[(int64_t)(case0 + c) * n + D.xrow[xb + x]] : 0.0;
    }
    if (tid < kPB) {                                    // line changes and losses of each case
        const int c = tid, k = case0 + c;
        const bool ok = c < nvc;
        cnt[c] = ok ? M.count[k] : 0;
        nlost[c] = ok ? E.loss_cnt[k] : 0;
        for (int j = 0; j < R; ++j) {
            mact[c * R + j] = ok ? M.act[k * R + j] : 0x7fffffff;
            mdg[c * R + j] = ok ? M.dg[k * R + j] : 0.0;
            lbr[c * R + j] = ok ? E.loss_br[k * R + j] : -1;
            lst[c * R + j] = ok ? E.loss_step[k * R + j] : 0x7fffffff;
            lpa[c * R + j] = D.lpa[((int64_t)tw * kPB + c) * R + j];
            lpb[c * R + j] = D.lpb[((int64_t)tw * kPB + c) * R + j];
            if (ok && j < M.count[k] && (lpa[c * R + j] < 0 || (M.b[k * R + j] >= 0 && lpb[c * R + j] < 0)))
                atomicOr(P.flags, kFlagTeamRow);
        }
        for (int i = 0; i < R * R * R; ++i) cinv[c * R * R * R + i] = ok ? M.Cinv[(int64_t)k * R * R * R + i] : 0.0;
    }
    // SMW vectors u_j of each case at own rows ([j][r][c]) and X rows ([j][x][c])
    for (int i = tid; i < R * NLp * kPB; i += kPThreads) {
        const int j = i / (NLp * kPB), rc = i - j * NLp * kPB, r = rc >> 4, c = rc & 15;
        TB u = 0;
        if (r < nl && c < nvc && j < M.count[case0 + c]) u = gU[((int64_t)(case0 + c) * R + j) * n + lo + r];
        uo[i] = u;
    }
    for (int i = tid; i < R * D.NX * kPB; i += kPThreads) {
        const int j = i / (D.NX * kPB), xc = i - j * D.NX * kPB, x = xc >> 4, c = xc & 15;
        TB u = 0;
        if (x < nx && c < nvc && j < M.count[case0 + c]) u = gU[((int64_t)(case0 + c) * R + j) * n + D.xrow[xb + x]];
        ux[i] = u;
    }
    // capacitor histories of the thread's (row, case) items, in registers
    double hcr[kPRowItems];
#pragma unroll
    for (int it = 0; it < kPRowItems; ++it) {
        const int i = tid + it * kPThreads, r = i >> 4, c = i & 15;
        hcr[it] = (r < nl && c < nvc) ? E.hC[(int64_t)(case0 + c) * n + lo + r] : 0.0;
    }
    // leaf block as A fragments (zero outside the leaf)
    const PanelGemm gm = panel_gemm(NLp);
    const bool gwave = wave < gm.MT * gm.KSPLIT;
    const int mt = wave % gm.MT, kp = wave / gm.MT;
    const int ks0 = kp * gm.KSC;
    int nks = 0;
    if (gwave) {
        const int e = ks0 + gm.KSC < gm.KS ? ks0 + gm.KSC : gm.KS;
        nks = e > ks0 ? e - ks0 : 0;
    }
    TB afrag[kPMaxFrag];
    {
        const TB* src = gblk + H.leaf_off[l];
        const int row = mt * 16 + (lane & 15);
#pragma unroll
        for (int f = 0; f < kPMaxFrag; ++f) {
            TB a = 0;
            const int col = (ks0 + f) * 4 + (lane >> 4);
            if (f < nks && row < nl && col < nl) a = src[(int64_t)col * nl + row];
            afrag[f] = a;
        }
    }
    __syncthreads();

    int par = 0;
    unsigned int epoch = 0;
    bool alive = true;
    double worst = 0.0;
    unsigned int* tflags = D.sync + (int64_t)team * T;
    const int NXs = D.NX;
    const int ns = sptr[nl];
    int64_t sn_step = -1;    // the step whose source injections the next apply computes (-1: none)

    // value of a combined row index (own row or X row) in the pair (own, X)
    auto cval = [&](const double* own, const double* xr, int comb, int c) -> double {
        return comb < nl ? own[comb * kPB + c] : xr[(comb - nl) * kPB + c];
    };

    // one application of the stored inverse with each case's active changes:
    // out (own rows), outx (X rows) from xin (own rows, zero beyond nl); out
    // may be xin (it is written after every wavefront has read xin)
    auto apply = [&](const double* xin, double* out, double* outx, bool anyact, bool want_vm) -> bool {
        double* X0p = D.X0 + ((int64_t)team * 2 + par) * (int64_t)n * kPB;
        const double* VMp = D.VM + ((int64_t)team * 2 + par) * T * kPB;
        {
            typename Mfma16<TB>::V acc = {0, 0, 0, 0};
#pragma unroll
            for (int f = 0; f < kPMaxFrag; ++f) {
                if (f < nks) {
                    const int k = (ks0 + f) * 4 + (lane >> 4);
                    acc = Mfma16<TB>::op(afrag[f], (TB)xin[k * kPB + (lane & 15)], acc);
                }
            }
            if (gwave && kp > 0) {
                double* pp = y + ((kp - 1) * gm.MT + mt) * 256;
#pragma unroll
                for (int i = 0; i < 4; ++i) pp[i * 64 + lane] = (double)acc[i];
            }
            __syncthreads();
            if (gwave && kp == 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    double val = (double)acc[i];
                    for (int q = 1; q < gm.KSPLIT; ++q) val += y[((q - 1) * gm.MT + mt) * 256 + i * 64 + lane];
                    const int r = mt * 16 + Mfma16<TB>::row(lane, i), c = lane & 15;
                    if (r < nl) {
                        out[r * kPB + c] = val;
                        xchg_store(&X0p[(int64_t)(lo + r) * kPB + c], val);
                    }
                }
            }
        }
        team_arrive(tflags, l, ++epoch);
        if (sn_step >= 0) {      // source injections of the next step, by the last wavefront, while wavefront 0 polls
            if (tid >= kPThreads - 64)
                for (int q = tid - (kPThreads - 64); q < ns; q += 64)
                    sn[q] = samp[q] * sin(E.omega * ((double)sn_step * E.dt) + sph[q]);
            sn_step = -1;
        }
        if (!team_wait(tflags, T, epoch, P.flags, ctl)) return false;
        if (want_vm) {   // the team's largest |v| per case (vg was cleared before the barrier)
            for (int i = tid; i < T * kPB; i += kPThreads)
                atomicMax(&vg[i & 15], (unsigned long long)__double_as_longlong(xchg_load(&VMp[i])));
        }
        {   // every load of the exchange is issued before the first wait
            double xl[kPXItems], cl[kPColItems];
#pragma unroll
            for (int it = 0; it < kPXItems; ++it) {
                const int i = tid + it * kPThreads;
                xl[it] = i < nx * kPB ? xchg_load(&X0p[(int64_t)xrow[i >> 4] * kPB + (i & 15)]) : 0.0;
            }
#pragma unroll
            for (int it = 0; it < kPColItems; ++it) {
                const int i = tid + it * kPThreads;
                cl[it] = i < nc * kPB ? xchg_load(&X0p[(int64_t)crow[i >> 4] * kPB + (i & 15)]) : 0.0;
            }
#pragma unroll
            for (int it = 0; it < kPXItems; ++it) {
                const int i = tid + it * kPThreads;
                if (i < nx * kPB) outx[i] = xl[it];
            }
#pragma unroll
            for (int it = 0; it < kPColItems; ++it) {
                const int i = tid + it * kPThreads;
                if (i < nc * kPB) y[i] = cl[it];
            }
        }
        __syncthreads();
        // coupling levels bottom-up; a level's slots of y hold the raw values,
        // then s = U^T v (lower-level corrections inline), then y = S^{-1} s
        for (int hl = 1; hl <= Hn; ++hl) {
            const int c0 = lvlc[hl - 1], c1 = lvlc[hl];
            if (c1 == c0) continue;
            for (int i = c0 * kPB + tid; i < c1 * kPB; i += kPThreads) {
                const int g = i >> 4, c = i & 15;
                double val = y[i];
                for (int hh = 1; hh < hl; ++hh) {
                    const int zo = czo[g * Hn + hh - 1];
                    if (zo >= 0) val -= (double)pdot<TA>(cz + zo, 1, y, cpc[g * Hn + hh - 1], cpm[g * Hn + hh - 1], c);
                }
                y[i] = colw[g] * val;
            }
            __syncthreads();
            // y = S^{-1} s on the matrix cores: every node's S^{-1} in 16-row tiles (zero beyond m)
            // times the node's s for the 16 cases, k-steps of 4; wavefront w takes the level's
            // tiles w and w + kPWaves (the host keeps a level at <= 2 * kPWaves tiles)
            {
                int tg[kPLevelTiles], tqt[kPLevelTiles];
#pragma unroll
                for (int k = 0; k < kPLevelTiles; ++k) tg[k] = -1;
                {
                    int tcount = 0;
                    for (int g = c0; g < c1; g += cm[g]) {
                        for (int qt = 0; qt * 16 < cm[g]; ++qt, ++tcount) {
#pragma unroll
                            for (int k = 0; k < kPLevelTiles; ++k)
                                if (tcount == wave + k * kPWaves) { tg[k] = g; tqt[k] = qt; }
                        }
                    }
                }
                typename Mfma16<TB>::V yacc[kPLevelTiles];
#pragma unroll
                for (int k = 0; k < kPLevelTiles; ++k) {
                    yacc[k] = typename Mfma16<TB>::V{0, 0, 0, 0};
                    if (tg[k] >= 0) {
                        const int g0 = __builtin_amdgcn_readfirstlane(tg[k]);
                        const int m = __builtin_amdgcn_readfirstlane(cm[g0]);
                        const TB* Si = sall + cso[g0];
                        const int q = tqt[k] * 16 + (lane & 15), qc = q < m ? q : m - 1;
                        // four k-steps per round: clamped loads first (zero outside the node's
                        // m x m block), then four dependent matrix products
                        for (int k0 = 0; k0 < m; k0 += 16) {
                            TB a[4], bb[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int pp = k0 + u * 4 + (lane >> 4), pc = pp < m ? pp : m - 1;
                                const TB a0 = Si[qc + pc * (m + 1)];
                                const TB b0 = (TB)y[(g0 + pc) * kPB + (lane & 15)];
                                a[u] = (q < m && pp < m) ? a0 : (TB)0;
                                bb[u] = pp < m ? b0 : (TB)0;
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u) yacc[k] = Mfma16<TB>::op(a[u], bb[u], yacc[k]);
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < kPLevelTiles; ++k) {
                    if (tg[k] >= 0) {
                        const int g0 = tg[k], m = cm[g0];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int q = tqt[k] * 16 + Mfma16<TB>::row(lane, e);
                            if (q < m) y[(g0 + q) * kPB + (lane & 15)] = (double)yacc[k][e];
                        }
                    }
                }
            }
            __syncthreads();
        }
        // own rows and X rows: v -= sum over levels of Z y (one dot-product order for every row, so
        // rows shared by two workgroups stay bitwise identical)
        if constexpr (sizeof(TB) == 8) {
            // own rows on the matrix cores, one 16-row tile per wavefront: the FP64 16x16x4 product
            // rounds as a chain of fused multiply-adds over k (measured bitwise on gfx950), which is
            // the chain the X-row loop below uses for the same rows in other workgroups
            if (wave < gm.MT) {
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
                    const int pm = __builtin_amdgcn_readfirstlane(opm[hh]), pc = opc[hh];
                    typename Mfma16<TB>::V acc = {0, 0, 0, 0};
                    for (int k0 = 0; k0 < pm; k0 += 4) {
                        const int j = k0 + (lane >> 4), jc = j < pm ? j : pm - 1;
                        const TB a0 = zown[zo + jc * nl + rc];
                        const TB b0 = (TB)y[(pc + jc) * kPB + c];
                        acc = Mfma16<TB>::op((ra_ < nl && j < pm) ? a0 : (TB)0, j < pm ? b0 : (TB)0, acc);
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) val[e] -= (double)acc[e];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = r0 + Mfma16<TB>::row(lane, e);
                    if (r < nl) out[r * kPB + c] = val[e];
                }
            }
        } else {
            for (int i = tid; i < nl * kPB; i += kPThreads) {
                const int r = i >> 4, c = i & 15;
                double val = out[i];
                for (int hh = 0; hh < Hn; ++hh) {
                    const int zo = ozo[hh];
                    if (zo >= 0) val -= (double)pdot<TA>(zown + zo + r, nl, y, opc[hh], opm[hh], c);
                }
                out[i] = val;
            }
        }
        for (int i = tid; i < nx * kPB; i += kPThreads) {
            const int x = i >> 4, c = i & 15;
            double val = outx[i];
            for (int hh = 0; hh < Hn; ++hh) {
                const int zo = xzo[x * Hn + hh];
                if (zo >= 0) val -= (double)pdot<TA>(xz + zo, 1, y, xpc[x * Hn + hh], xpm[x * Hn + hh], c);
            }
            outx[i] = val;
        }
        __syncthreads();
        if (anyact) {                                   // per-case SMW correction
            if (tid < kPB) {
                const int c = tid, ra = ract[c];
                for (int j = 0; j < ra; ++j) {
                    const int a = lpa[c * R + j], bb = lpb[c * R + j];
                    tz[c * 2 * R + j] = cval(out, outx, a, c) - (bb >= 0 ? cval(out, outx, bb, c) : 0.0);
                }
                if (ra > 0) {
                    const double* Ci = cinv + (int64_t)c * R * R * R + (ra - 1) * R * R;
                    for (int j = 0; j < ra; ++j) {
                        double acc = 0.0;
                        for (int q = 0; q < ra; ++q) acc += Ci[j * R + q] * tz[c * 2 * R + q];
                        tz[c * 2 * R + R + j] = acc;
                    }
                }
            }
            __syncthreads();
            for (int i = tid; i < nl * kPB; i += kPThreads) {
                const int c = i & 15, ra = ract[c];
                double acc = 0.0;
                for (int j = 0; j < ra; ++j) acc = pfma((double)uo[j * NLp * kPB + i], tz[c * 2 * R + R + j], acc);
                out[i] -= acc;
            }
            for (int i = tid; i < nx * kPB; i += kPThreads) {
                const int c = i & 15, ra = ract[c];
                double acc = 0.0;
                for (int j = 0; j < ra; ++j) acc = pfma((double)ux[j * NXs * kPB + i], tz[c * 2 * R + R + j], acc);
                outx[i] -= acc;
            }
            __syncthreads();
        }
        par ^= 1;
        return true;
    };

    // t = b - G_step v on own rows (FP64), then v += P t; stats on the last pass
    auto refine = [&](bool anyact, bool last) -> bool {
        for (int i = tid; i < nl * kPB; i += kPThreads) {
            const int r = i >> 4, c = i & 15;
            double acc = 0.0;
            for (int e = orp[r]; e < orp[r + 1]; ++e) acc += oval[e] * cval(v, xv, ocol[e], c);
            const int ra = ract[c];
            for (int j = 0; j < ra; ++j) {
                const int a = lpa[c * R + j], bb = lpb[c * R + j];
                if (a != r && bb != r) continue;
                const double wv = cval(v, xv, a, c) - (bb >= 0 ? cval(v, xv, bb, c) : 0.0);
                acc += (a == r ? 1.0 : -1.0) * mdg[c * R + j] * wv;
            }
            td[i] = b[i] - acc;
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
        if (!MIXED && rec && P.b_rec) {                 // b is overwritten by v below
            for (int i = tid; i < nl * kPB; i += kPThreads) {
                const int c = i & 15;
                if (c < nvc) P.b_rec[(jr * K + case0 + c) * (int64_t)n + prow[i >> 4]] = b[i];
            }
        }
        if (tid < kPB) {
            int ra = 0;
            while (ra < cnt[tid] && (int64_t)mact[tid * R + ra] <= step) ++ra;
            ract[tid] = ra;
        }
        __syncthreads();
        bool anyact = false;
        for (int c = 0; c < kPB; ++c) anyact |= ract[c] > 0;
        if constexpr (!MIXED) {
            alive = apply(b, v, xv, anyact, false);
            applies += 1;
        } else {
            const int nref = WARM ? P.max_refine + 1 : P.max_refine;
            if (!WARM) {
                alive = apply(b, v, xv, anyact, false);
                applies += 1;
            }
            for (int q = 0; q < nref && alive; ++q) {
                alive = refine(anyact, q == nref - 1);
                applies += 1;
            }
        }
        if (!alive) break;
        // history: new branch histories, then the right-hand side of step+1
        for (int i = tid; i < nb * kPB; i += kPThreads) {
            const int q = i >> 4, c = i & 15;
            const int e = bglob[q];
            bool lost = false;
            for (int j = 0; j < nlost[c]; ++j)
                if (lbr[c * R + j] == e && (int64_t)lst[c * R + j] <= step + 1) lost = true;
            double hv = 0.0;
            if (!lost) {
                const double vft = cval(v, xv, bf[q], c) - cval(v, xv, bt[q], c);
                const double ie = bg[q] * vft + h[i];
                hv = bg[q] * vft + bal[q] * ie;
            }
            h[i] = hv;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPRowItems; ++k) {
            const int i = tid + k * kPThreads, r = i >> 4, c = i & 15;
            if (r < nl) {
                const double va = v[i];
                double bn = 0.0;
                for (int q = sptr[r]; q < sptr[r + 1]; ++q) bn += sn[q];
                for (int q = iptr[r]; q < iptr[r + 1]; ++q) {
                    const int lb = ibr[q];
                    const double hv = h[lb * kPB + c];
                    bn -= (bf[lb] == r) ? hv : -hv;
                }
                const double ic = gC[r] * va + hcr[k];
                const double hcn = -gC[r] * va - ic;
                hcr[k] = hcn;
                bn -= hcn;
                if (rec && c < nvc) {
                    const int64_t o = (jr * K + case0 + c) * (int64_t)n + prow[r];
                    if (P.v_rec) P.v_rec[o] = va;
                    if (MIXED && P.b_rec) P.b_rec[o] = b[i];
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
        if (c < nvc && D.bown[(int64_t)l * D.NB + q]) hdst[(int64_t)(case0 + c) * E.nbr + bglob[q]] = h[i];
    }
    if (tid < nvc) {
        if (MIXED && P.stats) atomicMax(&P.stats[case0 + tid], (unsigned long long)__double_as_longlong(worst));
        if (l == 0 && P.applies) atomicAdd(&P.applies[case0 + tid], (unsigned long long)applies);
    }
    if (blockIdx.x == 0 && tid == 0) *E.step = nstep;
}

template <typename TB, bool MIXED, bool WARM>
static hipError_t launch_panel_t(const PanelDev& D, const EmtDev& E, const HierDev& H, const ModDev& M,
                                 const RunParams& P, hipStream_t s)
{
    const size_t lds = panel_layout<TB, MIXED>(D, M.R).total;
    const void* fn = (const void*)k_emt_panel<TB, MIXED, WARM>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0, per = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kPThreads, lds);
    if (e != hipSuccess) return e;
    const int teams_per_launch = (per * cus) / D.T;     // teams that are co-resident in one launch
    if (teams_per_launch < 1) return hipErrorCooperativeLaunchTooLarge;
    e = hipMemsetAsync(D.sync, 0, (size_t)D.n_teams * D.T * sizeof(unsigned int), s);
    if (e != hipSuccess) return e;
    for (int t0 = 0; t0 < D.n_teams; t0 += teams_per_launch) {
        const int nt = D.n_teams - t0 < teams_per_launch ? D.n_teams - t0 : teams_per_launch;
        PanelDev Dc = D;
        Dc.team0 = t0;
        EmtDev Ec = E;
        HierDev Hc = H;
        ModDev Mc = M;
        RunParams Pc = P;
        void* args[] = {&Dc, &Ec, &Hc, &Mc, &Pc};
        e = hipLaunchCooperativeKernel(fn, dim3(nt * D.T), dim3(kPThreads), args, (unsigned int)lds, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_emt_panel(const PanelDev& D, const EmtDev& E, const HierDev& H, const ModDev& M, const RunParams& P,
                            int prec, hipStream_t s)
{
    if (prec == HINV_FP64) return launch_panel_t<double, false, false>(D, E, H, M, P, s);
    if (P.warm) return launch_panel_t<float, true, true>(D, E, H, M, P, s);
    return launch_panel_t<float, true, false>(D, E, H, M, P, s);
}

}  // namespace hinv
