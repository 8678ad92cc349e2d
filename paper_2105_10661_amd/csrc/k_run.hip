// Fused EMT stepping: one workgroup owns one case and advances it through
// all requested time steps in a single launch (paper Section II, Eq. (1)-(2)
// per step; Section IV's line change as the SMW correction).
//
// Per step, inside the workgroup:
//   apply        v0 = B^{-1} x leaf by leaf, then every coupling level bottom-up
//                (s = U^T v, y = S^{-1} s, v -= Z y), then the active line
//                changes v -= U_m C_m^{-1} (U_m^T x) (U_m = G0^{-1} W_m, so U_m^T x
//                equals W_m^T G0^{-1} x, taken from the input x);
//   refinement   (low-precision storage) t = b - G v in FP64, v += P t, until the
//                correction is below rel_tol * |v| or max_refine corrections;
//                optionally warm-started from the previous step's v; FP64 storage
//                warm-started is the incremental form, one pass v += P (b - G v);
//   history      trapezoidal history currents with v_n and b_{n+1}.
// The case's vectors b (right-hand side), v (solution), t (residual) and d
// (correction) live in LDS for the whole launch; the stored
// inverse (shared by all cases of the network) streams from L2.  Nothing is
// exchanged between workgroups, so the same kernel runs one case or a batch
// (one workgroup per case), and every case's arithmetic is independent of the
// batch it runs in.
//
// Thread layout (1024 threads): one thread per row in the leaf apply (a
// wavefront reads 64 consecutive rows of a block column per load), one thread
// per coupling column or panel row in the level phases.
#include "hinv_internal.h"

namespace hinv {

constexpr int kRunThreads = 1024;

template <typename TB>
struct Acc { using T = float; };
template <>
struct Acc<double> { using T = double; };

__device__ inline double block_max(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double m = red[0];
    for (int w = 1; w < kRunThreads / 64; ++w) m = fmax(m, red[w]);
    __syncthreads();
    return m;
}

// out = B^{-1} x over all leaves (x, out: distinct LDS vectors).  One thread
// per row; a wavefront covers 64 consecutive rows, so every load instruction
// reads one contiguous run of a block column.  Loads are issued in batches of
// kBatch before they are consumed, to keep many requests in flight per CU.
template <typename TB>
__device__ void wg_leaf_apply(const HierDev& H, const TB* __restrict__ blk, const double* x, double* out)
{
    using TA = typename Acc<TB>::T;
    constexpr int kBatch = 16;
    for (int r = threadIdx.x; r < H.n; r += kRunThreads) {
        const int lo = H.row_lo[r], nl = H.row_nl[r];
        const TB* Bp = blk + H.row_boff[r];
        const double* xl = x + lo;
        TA acc = 0;
        for (int j0 = 0; j0 < nl; j0 += kBatch) {
            TB bv[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) bv[q] = (j0 + q < nl) ? Bp[(int64_t)(j0 + q) * nl] : (TB)0;
#pragma unroll
            for (int q = 0; q < kBatch; ++q)
                if (j0 + q < nl) acc += (TA)bv[q] * (TA)xl[j0 + q];
        }
        out[r] = (double)acc;
    }
    __syncthreads();
}

// Coupling levels bottom-up on out (LDS).  s, y: LDS scratch of n_cols.
template <typename TB>
__device__ void wg_levels(const HierDev& H, const TB* __restrict__ Z, const TB* __restrict__ Sinv, double* out,
                          double* s, double* y)
{
    using TA = typename Acc<TB>::T;
    const int tid = threadIdx.x;
    for (int h = 1; h <= H.n_levels; ++h) {
        const int c0 = H.lvl_col[h - 1], c1 = H.lvl_col[h];
        if (c1 == c0) continue;
        for (int g = c0 + tid; g < c1; g += kRunThreads) s[g] = H.col_w[g] * out[H.col_row[g]];
        __syncthreads();
        for (int g = c0 + tid; g < c1; g += kRunThreads) {
            const int m = H.col_m[g], nc0 = H.col_c0[g];
            const TB* Si = Sinv + H.col_soff[g];
            TA acc = 0;
            for (int pp = 0; pp < m; ++pp) acc += (TA)Si[(int64_t)pp * m] * (TA)s[nc0 + pp];
            y[g] = (double)acc;
        }
        __syncthreads();
        const int f0 = H.lvl_frow[h - 1], f1 = H.lvl_frow[h];
        for (int f = f0 + tid; f < f1; f += kRunThreads) {
            const int pn = H.frow_pn[f], pm = H.frow_pm[f], pc0 = H.frow_pc[f];
            const TB* Zp = Z + H.frow_z[f];
            TA acc = 0;
            for (int j = 0; j < pm; ++j) acc += (TA)Zp[(int64_t)j * pn] * (TA)y[pc0 + j];
            out[H.frow_row[f]] -= (double)acc;
        }
        __syncthreads();
    }
}

// Active line changes of case k at `step` on out (LDS); x is the apply's input.  Each change's
// coefficient is t_j = u_j^T x with u_j = G0^{-1} w_j (G0 symmetric: the same as w_j^T G0^{-1} x), taken
// from x rather than from the apply's values at the change's endpoints, which carry the stored
// inverse's rounding (FP32 storage: ~1e-7 relative) into a term that the capacitance's inverse
// amplifies when the change nearly separates the network (a bus left on its shunt capacitor).  The
// sum over rows is a fixed tree (per wavefront, then the wavefronts in order): red holds one value per
// wavefront.
template <typename TU>
__device__ void wg_smw(const ModDev& M, const TU* __restrict__ U, int k, int64_t step, const double* x, double* out,
                       double* tz, double* red)
{
    const int cnt = M.count[k];
    int r = 0;
    while (r < cnt && (int64_t)M.act[k * M.R + r] <= step) ++r;
    if (r == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int j = 0; j < r; ++j) {
        const TU* u = U + ((int64_t)k * M.R + j) * M.n;
        double acc = 0.0;
        for (int i = tid; i < M.n; i += kRunThreads) acc = fma((double)u[i], x[i], acc);
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) red[wave] = acc;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < kRunThreads / 64; ++w) sum += red[w];
            tz[j] = sum;
        }
        __syncthreads();
    }
    if (tid < r) {
        const double* Ci = M.Cinv + ((int64_t)k * M.R + (r - 1)) * M.R * M.R;
        double acc = 0.0;
        for (int j = 0; j < r; ++j) acc += Ci[tid * M.R + j] * tz[j];
        tz[kMaxModRank + tid] = acc;
    }
    __syncthreads();
    for (int i = tid; i < M.n; i += kRunThreads) {
        double acc = 0.0;
        for (int j = 0; j < r; ++j) acc += (double)U[((int64_t)k * M.R + j) * M.n + i] * tz[kMaxModRank + j];
        out[i] -= acc;
    }
    __syncthreads();
}

template <typename TB>
__device__ void wg_precond(const HierDev& H, const ModDev& M, const TB* blk, const TB* Z, const TB* Sinv,
                           const TB* U, int k, int64_t step, const double* x, double* out, double* s, double* y,
                           double* tz, double* red)
{
    wg_leaf_apply<TB>(H, blk, x, out);
    wg_levels<TB>(H, Z, Sinv, out, s, y);
    if (M.R > 0) wg_smw<TB>(M, U, k, step, x, out, tz, red);
}

// t = b - G_step v (FP64, LDS vectors).
__device__ void wg_residual(const HierDev& H, const ModDev& M, int k, int64_t step, const double* b, const double* v,
                            double* t)
{
    int r = 0;
    if (M.R > 0) {
        const int cnt = M.count[k];
        while (r < cnt && (int64_t)M.act[k * M.R + r] <= step) ++r;
    }
    for (int i = threadIdx.x; i < H.n; i += kRunThreads) {
        double acc = 0.0;
        for (int e = H.rp[i]; e < H.rp[i + 1]; ++e) acc += H.cv[e] * v[H.ci[e]];
        for (int j = 0; j < r; ++j) {
            const int a = M.a[k * M.R + j], bb = M.b[k * M.R + j];
            if (i != a && i != bb) continue;
            if (M.grp3) {          // row j of the line's 3x3 D times its three phase differences
                const int g0 = j - j % 3;
                const double* dj = M.d3 + ((int64_t)k * M.R + j) * 3;
                double dw = 0.0;
                for (int q = 0; q < 3; ++q) {
                    const int aq = M.a[k * M.R + g0 + q], bq = M.b[k * M.R + g0 + q];
                    dw += dj[q] * (v[aq] - (bq >= 0 ? v[bq] : 0.0));
                }
                acc += (i == a ? 1.0 : -1.0) * dw;
                continue;
            }
            const double wv = v[a] - (bb >= 0 ? v[bb] : 0.0);
            acc += (i == a ? 1.0 : -1.0) * M.dg[k * M.R + j] * wv;
        }
        t[i] = b[i] - acc;
    }
    __syncthreads();
}

__device__ inline bool run_lost_by(const EmtDev& E, int k, int e, int64_t step)
{
    const int cnt = E.loss_cnt[k];
    for (int j = 0; j < cnt; ++j)
        if (E.loss_br[k * E.R + j] == e && (int64_t)E.loss_step[k * E.R + j] <= step) return true;
    return false;
}

// The whole per-case stepping loop; b, v, t, d are LDS (or, for cases too big
// for LDS, the case's global scratch), s, y, red, tz are LDS.  MIXED with FP64
// storage is the incremental form v = v_prev + P (b - G v_prev): one FP64
// apply per step, no convergence test (P is the FP64 inverse).
template <typename TB, bool MIXED, bool WARM>
__device__ __forceinline__ void emt_run_body(const EmtDev& E, const HierDev& H, const ModDev& M, const RunParams& P,
                                             int k, double* b, double* v, double* t, double* d, double* s, double* y,
                                             double* red, double* tz)
{
    constexpr bool INC = MIXED && sizeof(TB) == 8;
    static_assert(!INC || WARM, "the incremental FP64 form starts from the previous step's voltages");
    const int n = H.n;
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)k * n;
    const TB* blk;
    const TB* Zs;
    const TB* Si;
    const TB* U;
    if constexpr (sizeof(TB) == 8) {
        blk = (const TB*)H.blk; Zs = (const TB*)H.Z; Si = (const TB*)H.Sinv; U = (const TB*)M.U;
    } else {
        blk = (const TB*)H.blk32; Zs = (const TB*)H.Z32; Si = (const TB*)H.Sinv32; U = (const TB*)M.U32;
    }
    for (int i = tid; i < n; i += kRunThreads) {
        b[i] = E.b[base + i];
        v[i] = E.v[base + i];
    }
    __syncthreads();
    double worst = 0.0;
    int64_t applies = 0;
    for (int it = 0; it < P.n_steps; ++it) {
        const int64_t step = P.step0 + it;
        // ---- solve G_step v = b
        if (!MIXED) {
            wg_precond<TB>(H, M, blk, Zs, Si, U, k, step, b, v, s, y, tz, red);
            applies += 1;
        } else {
            int done = 0;
            if (!WARM) {
                wg_precond<TB>(H, M, blk, Zs, Si, U, k, step, b, v, s, y, tz, red);
                applies += 1;
            }
            const int nref = INC ? 1 : P.max_refine + (WARM ? 1 : 0);
            for (int rf = 0; rf < nref && !done; ++rf) {
                wg_residual(H, M, k, step, b, v, t);
                wg_precond<TB>(H, M, blk, Zs, Si, U, k, step, t, d, s, y, tz, red);
                applies += 1;
                if constexpr (INC) {
                    for (int i = tid; i < n; i += kRunThreads) v[i] += d[i];
                    __syncthreads();
                    continue;
                }
                double dmax = 0.0, vmax = 0.0;
                for (int i = tid; i < n; i += kRunThreads) {
                    const double nv = v[i] + d[i];
                    v[i] = nv;
                    dmax = fmax(dmax, fabs(d[i]));
                    vmax = fmax(vmax, fabs(nv));
                }
                dmax = block_max(dmax, red);
                vmax = block_max(vmax, red);
                const double ratio = vmax > 0.0 ? dmax / vmax : (dmax > 0.0 ? INFINITY : 0.0);
                if (!isfinite(ratio)) {
                    if (tid == 0) atomicOr(P.flags, kFlagNaN);
                    done = 1;
                } else if (ratio <= P.rel_tol) {
                    done = 1;
                    worst = fmax(worst, ratio);
                } else if (rf == nref - 1) {
                    if (tid == 0) atomicOr(P.flags, kFlagNoConv);
                    worst = fmax(worst, ratio);
                }
            }
        }
        // ---- history update with v_step, right-hand side of step+1, records
        const double* hcur = E.h + (int64_t)(step & 1) * E.n_cases * E.nbr + (int64_t)k * E.nbr;
        double* hnext = E.h + (int64_t)((step + 1) & 1) * E.n_cases * E.nbr + (int64_t)k * E.nbr;
        const int64_t j = step - P.step0;
        for (int a = tid; a < n; a += kRunThreads) {
            const double va = v[a];
            double bn = 0.0;
            for (int q = E.src_ptr[a]; q < E.src_ptr[a + 1]; ++q)
                bn += E.src_amp[q] * sin(E.omega * ((double)(step + 1) * E.dt) + E.src_ph[q]);
            for (int q = E.inc_ptr[a]; q < E.inc_ptr[a + 1]; ++q) {
                const int e = E.inc_br[q];
                const int f = E.fr[e], to = E.to[e];
                double hn = 0.0;
                if (!run_lost_by(E, k, e, step + 1)) {
                    if (E.Y3) {        // three-phase: phase e % 3 of line e / 3
                        hn = line3_history(E, v, hcur, e / 3, e % 3);
                    } else {
                        const double vft = v[f] - v[to];
                        const double ie = E.g[e] * vft + hcur[e];
                        hn = E.g[e] * vft + E.alpha[e] * ie;
                    }
                }
                bn -= (a == f) ? hn : -hn;
                if (a == f) hnext[e] = hn;
            }
            const double ic = E.gC[a] * va + E.hC[base + a];
            const double hcn = -E.gC[a] * va - ic;
            E.hC[base + a] = hcn;
            bn -= hcn;
            const int64_t jr = step - P.rec_step0;
            if (jr >= 0 && jr < P.rec_cap) {
                const int64_t o = (jr * E.n_cases + k) * (int64_t)n + E.perm[a];
                if (P.v_rec) P.v_rec[o] = va;
                if (P.b_rec) P.b_rec[o] = b[a];
            }
            b[a] = bn;
        }
        __syncthreads();
        if (P.clk && k == 0 && tid == 0 && j < P.clk_cap) P.clk[j] = (int64_t)wall_clock64();
    }
    for (int i = tid; i < n; i += kRunThreads) {
        E.b[base + i] = b[i];
        E.v[base + i] = v[i];
    }
    if (tid == 0) {
        if (MIXED && !INC && P.stats) atomicMax(&P.stats[k], (unsigned long long)__double_as_longlong(worst));
        if (P.applies) atomicAdd(&P.applies[k], (unsigned long long)applies);
        if (k == 0) *E.step = P.step0 + P.n_steps;
    }
}

template <typename TB, bool MIXED, bool WARM>
__global__ __launch_bounds__(kRunThreads) void k_emt_run(EmtDev E, HierDev H, ModDev M, RunParams P)
{
    extern __shared__ double lds[];
    const int n = H.n;
    double* b = lds;
    double* v = b + n;
    double* t = v + n;
    double* d = t + n;
    double* s = d + n;
    double* y = s + H.n_cols;
    double* red = y + H.n_cols;          // 16
    double* tz = red + 16;               // 2 * kMaxModRank
    emt_run_body<TB, MIXED, WARM>(E, H, M, P, blockIdx.x, b, v, t, d, s, y, red, tz);
}

// Serving: one workgroup per slot; every slot is its own case (own network,
// hierarchy and state); the start step comes from the case's step counter.
template <typename TB, bool MIXED, bool WARM>
__global__ __launch_bounds__(kRunThreads) void k_emt_serve(const ServeSlot* __restrict__ slots, int n_steps)
{
    extern __shared__ double lds[];
    __shared__ ServeSlot sl;
    __shared__ RunParams P;
    if (threadIdx.x == 0) {
        sl = slots[blockIdx.x];
        P.step0 = __hip_atomic_load(sl.E.step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.n_steps = n_steps;
        P.max_refine = sl.max_refine;
        P.rel_tol = sl.rel_tol;
        P.warm = WARM ? 1 : 0;
        P.v_rec = sl.v_rec;
        P.b_rec = nullptr;
        P.rec_step0 = sl.rec_step0;
        P.rec_cap = sl.rec_cap;
        P.flags = sl.flags;
        P.stats = sl.stats;
        P.applies = sl.applies;
        P.clk = nullptr;
        P.clk_cap = 0;
    }
    __syncthreads();
    const int n = sl.H.n;
    double* s = lds;
    double* y = s + sl.H.n_cols;
    double* red = y + sl.H.n_cols;
    double* tz = red + 16;
    if (sl.gvec) {
        double* g = sl.gscr;
        emt_run_body<TB, MIXED, WARM>(sl.E, sl.H, sl.M, P, sl.k, g, g + n, g + 2 * n, g + 3 * n, s, y, red, tz);
    } else {
        double* vb = tz + 2 * kMaxModRank;
        emt_run_body<TB, MIXED, WARM>(sl.E, sl.H, sl.M, P, sl.k, vb, vb + n, vb + 2 * n, vb + 3 * n, s, y, red, tz);
    }
}

size_t run_lds_bytes(const HierDev& H)
{
    return sizeof(double) * (4 * (size_t)H.n + 2 * (size_t)H.n_cols + 16 + 2 * kMaxModRank);
}

bool run_fits(const HierDev& H) { return run_lds_bytes(H) <= 160 * 1024; }

template <typename TB, bool MIXED, bool WARM>
static hipError_t launch_run_t(const EmtDev& E, const HierDev& H, const ModDev& M, const RunParams& P, hipStream_t s)
{
    const size_t lds = run_lds_bytes(H);
    hipError_t e = hipFuncSetAttribute((const void*)k_emt_run<TB, MIXED, WARM>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_emt_run<TB, MIXED, WARM>), dim3(E.n_cases), dim3(kRunThreads), lds, s, E, H, M, P);
    return hipGetLastError();
}

size_t serve_lds_bytes(const HierDev& H, bool gvec)
{
    return sizeof(double) * ((gvec ? 0 : 4 * (size_t)H.n) + 2 * (size_t)H.n_cols + 16 + 2 * kMaxModRank);
}

template <typename TB, bool MIXED, bool WARM>
static hipError_t launch_serve_t(const ServeSlot* slots, int n_slots, int n_steps, size_t lds, hipStream_t s)
{
    hipError_t e = hipFuncSetAttribute((const void*)k_emt_serve<TB, MIXED, WARM>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_emt_serve<TB, MIXED, WARM>), dim3(n_slots), dim3(kRunThreads), lds, s, slots, n_steps);
    return hipGetLastError();
}

hipError_t launch_emt_serve(const ServeSlot* d_slots, int n_slots, int n_steps, size_t lds, int prec, int warm,
                            hipStream_t s)
{
    if (n_slots <= 0) return hipSuccess;
    if (prec == HINV_FP64)
        return warm ? launch_serve_t<double, true, true>(d_slots, n_slots, n_steps, lds, s)
                    : launch_serve_t<double, false, false>(d_slots, n_slots, n_steps, lds, s);
    if (warm) return launch_serve_t<float, true, true>(d_slots, n_slots, n_steps, lds, s);
    return launch_serve_t<float, true, false>(d_slots, n_slots, n_steps, lds, s);
}

hipError_t launch_emt_run(const EmtDev& E, const HierDev& H, const ModDev& M, const RunParams& P, int prec,
                          hipStream_t s)
{
    if (prec == HINV_FP64)
        return P.warm ? launch_run_t<double, true, true>(E, H, M, P, s) : launch_run_t<double, false, false>(E, H, M, P, s);
    if (P.warm) return launch_run_t<float, true, true>(E, H, M, P, s);
    return launch_run_t<float, true, false>(E, H, M, P, s);
}

}  // namespace hinv
