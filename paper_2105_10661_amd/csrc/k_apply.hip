// Per-step apply of the stored exact inverse (paper Eq. (2): v = G^{-1} i),
// bottom-up over the partition tree, plus the line-change correction and the
// FP64 residual used by iterative refinement.
//
//  leaf_apply   : v0_l = B_l^{-1} i_l for every leaf (batched dense GEMV;
//                 lanes own rows so block columns stream coalesced, the four
//                 waves of a block split the columns, partial sums meet in LDS).
//  level_solve  : per internal node t: s = U_t^T v (gathers at the cut-line
//                 endpoints), y = S_t^{-1} s.
//  level_update : per child panel: v[rows(c)] -= Z_{t,c} y[cols(c)].
//                 Level by level, so level l reads the result of level l-1.
//                 For one node this is G_t^{-1} = B^{-1} - Z S^{-1} Z^T
//                 (Woodbury), the exact form of the paper's Eq. (8)-(9).
//  smw_apply    : v = v0 - U_m C_m^{-1} (W_m^T v0) for the line changes that
//                 are active (Sherman-Morrison-Woodbury; Section IV's problem).
//  residual     : r = i - G v in FP64 from the sparse G plus the active changes.
//
// Storage precision TB (double or float) with accumulator TA (double for
// double storage, float otherwise); vectors stay FP64 in memory.
#include "hinv_internal.h"

namespace hinv {

template <typename S, typename TA>
__global__ __launch_bounds__(kBlock) void k_leaf_apply(HierDev H, S blk, const double* __restrict__ X,
                                                        double* __restrict__ Xo)
{
    __shared__ TA xs[kMaxLeaf];
    __shared__ TA part[kBlock / 64][kMaxLeaf];
    const int l = blockIdx.x;
    const int64_t col = (int64_t)blockIdx.y * H.n;
    const int lo = H.leaf_lo[l], nl = H.leaf_n[l];
    const int64_t B = H.leaf_off[l];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int i = tid; i < nl; i += kBlock) xs[i] = (TA)X[col + lo + i];
    __syncthreads();
    for (int r = lane; r < nl; r += 64) {
        TA acc = 0;
        for (int j = wave; j < nl; j += kBlock / 64) acc += (TA)blk[B + j * nl + r] * xs[j];
        part[wave][r] = acc;
    }
    __syncthreads();
    for (int r = tid; r < nl; r += kBlock) {
        TA acc = part[0][r];
        for (int w = 1; w < kBlock / 64; ++w) acc += part[w][r];
        Xo[col + lo + r] = (double)acc;
    }
}

template <typename S, typename TA>
__global__ __launch_bounds__(kBlock) void k_level_solve(HierDev H, S Sinv, int level, const double* __restrict__ X,
                                                         double* __restrict__ Y)
{
    extern __shared__ unsigned char shraw[];
    TA* s = reinterpret_cast<TA*>(shraw);
    const int t = H.lvl_node[level - 1] + blockIdx.x;
    const int64_t xc = (int64_t)blockIdx.y * H.n;
    const int64_t yc = (int64_t)blockIdx.y * H.n_cols;
    const int m = H.node_m[t], c0 = H.node_col0[t];
    const int64_t Si = H.node_soff[t];
    for (int q = threadIdx.x; q < m; q += kBlock) s[q] = (TA)(H.col_w[c0 + q] * X[xc + H.col_row[c0 + q]]);
    __syncthreads();
    for (int q = threadIdx.x; q < m; q += kBlock) {
        TA acc = 0;
        for (int j = 0; j < m; ++j) acc += (TA)Sinv[Si + (int64_t)j * m + q] * s[j];
        Y[yc + c0 + q] = (double)acc;
    }
}

template <typename S, typename TA>
__global__ __launch_bounds__(kBlock) void k_level_update(HierDev H, S Z, int level, double* __restrict__ X,
                                                          const double* __restrict__ Y)
{
    extern __shared__ unsigned char shraw[];
    TA* y = reinterpret_cast<TA*>(shraw);
    const int P = H.lvl_pan[level - 1] + blockIdx.x;
    const int64_t xc = (int64_t)blockIdx.z * H.n;
    const int64_t yc = (int64_t)blockIdx.z * H.n_cols;
    const int plo = H.pan_lo[P], pn = H.pan_n[P], pm = H.pan_m[P], pc0 = H.pan_col0[P];
    const int64_t Zp = H.pan_zoff[P];
    for (int j = threadIdx.x; j < pm; j += kBlock) y[j] = (TA)Y[yc + pc0 + j];
    __syncthreads();
    const int i = blockIdx.y * kBlock + threadIdx.x;
    if (i < pn) {
        TA acc = 0;
        for (int j = 0; j < pm; ++j) acc += (TA)Z[Zp + (int64_t)j * pn + i] * y[j];
        X[xc + plo + i] -= (double)acc;
    }
}

template <typename S, typename TA>
static void apply_t(const HierDev& H, const LevelHost* lv, S blk, S Z, S Sinv, const double* X, double* Xo, double* Y,
                    int nrhs, hipStream_t s)
{
    hipLaunchKernelGGL((k_leaf_apply<S, TA>), dim3(H.n_leaves, nrhs), dim3(kBlock), 0, s, H, blk, X, Xo);
    for (int l = 1; l <= H.n_levels; ++l) {
        const LevelHost& L = lv[l - 1];
        if (L.nnodes == 0 || L.ncols == 0) continue;
        hipLaunchKernelGGL((k_level_solve<S, TA>), dim3(L.nnodes, nrhs), dim3(kBlock), sizeof(TA) * L.max_m, s, H,
                           Sinv, l, (const double*)Xo, Y);
        const int gy = (L.max_pan_rows + kBlock - 1) / kBlock;
        hipLaunchKernelGGL((k_level_update<S, TA>), dim3(L.npan, gy, nrhs), dim3(kBlock), sizeof(TA) * L.max_m, s, H,
                           Z, l, Xo, (const double*)Y);
    }
}

void launch_apply(const HierDev& H, const LevelHost* lv, int prec, const double* X, double* Xout, double* Y,
                  int nrhs, hipStream_t s)
{
    if (nrhs <= 0) return;
    switch (prec) {
    case HINV_FP64:
        apply_t<StF64, double>(H, lv, StF64{H.blk}, StF64{H.Z}, StF64{H.Sinv}, X, Xout, Y, nrhs, s);
        break;
    case HINV_FP32:
        apply_t<StF32, float>(H, lv, StF32{H.blk32}, StF32{H.Z32}, StF32{H.Sinv32}, X, Xout, Y, nrhs, s);
        break;
    case HINV_BF16:
        apply_t<StBF16, float>(H, lv, StBF16{H.blk16}, StBF16{H.Z16}, StBF16{H.Sinv16}, X, Xout, Y, nrhs, s);
        break;
    default:
        apply_t<StFP8, float>(H, lv, StFP8{H.blk8, H.blk8s}, StFP8{H.Z8, H.Z8s}, StFP8{H.Sinv8, H.Sinv8s}, X, Xout, Y,
                              nrhs, s);
        break;
    }
}

// ----------------------------------------------------------------------------
__global__ void k_permute_in(int n, int nrhs, const int* __restrict__ perm, const double* __restrict__ src, int ld,
                             double* __restrict__ X)
{
    const int64_t tot = (int64_t)n * nrhs;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(idx / n), r = (int)(idx - (int64_t)k * n);
        X[idx] = src[(int64_t)k * ld + perm[r]];
    }
}

__global__ void k_permute_out(int n, int nrhs, const int* __restrict__ perm, const double* __restrict__ X,
                              double* __restrict__ dst, int ld)
{
    const int64_t tot = (int64_t)n * nrhs;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(idx / n), r = (int)(idx - (int64_t)k * n);
        dst[(int64_t)k * ld + perm[r]] = X[idx];
    }
}

static int grid_for(int64_t tot)
{
    int64_t g = (tot + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (int)g;
}

void launch_permute_in(int n, int nrhs, const int* perm, const double* src, int ld, double* X, hipStream_t s)
{
    hipLaunchKernelGGL(k_permute_in, dim3(grid_for((int64_t)n * nrhs)), dim3(kBlock), 0, s, n, nrhs, perm, src, ld, X);
}

void launch_permute_out(int n, int nrhs, const int* perm, const double* X, double* dst, int ld, hipStream_t s)
{
    hipLaunchKernelGGL(k_permute_out, dim3(grid_for((int64_t)n * nrhs)), dim3(kBlock), 0, s, n, nrhs, perm, X, dst, ld);
}

// ----------------------------------------------------------------------------
// Number of changes of set k active at `step` (activation steps are sorted).
__device__ inline int active_count(const ModDev& M, int set, const int64_t* step_ptr)
{
    const int cnt = M.count[set];
    if (!step_ptr) return cnt;
    const int64_t st = *step_ptr;
    int r = 0;
    while (r < cnt && (int64_t)M.act[set * M.R + r] <= st) ++r;
    return r;
}

template <typename TU>
__global__ __launch_bounds__(kBlock) void k_smw_apply(ModDev M, const TU* __restrict__ U, double* __restrict__ V,
                                                       int set0, int set_stride, const int64_t* step_ptr)
{
    __shared__ double z[kMaxModRank];
    const int k = blockIdx.y, set = set0 + k * set_stride;
    const int r = active_count(M, set, step_ptr);
    if (r == 0) return;
    double* v = V + (int64_t)k * M.n;
    if (threadIdx.x == 0) {
        double t[kMaxModRank];
        for (int j = 0; j < r; ++j) {
            const int a = M.a[set * M.R + j], b = M.b[set * M.R + j];
            t[j] = v[a] - (b >= 0 ? v[b] : 0.0);
        }
        const double* Ci = M.Cinv + ((int64_t)set * M.R + (r - 1)) * M.R * M.R;
        for (int i = 0; i < r; ++i) {
            double acc = 0.0;
            for (int j = 0; j < r; ++j) acc += Ci[i * M.R + j] * t[j];
            z[i] = acc;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < M.n; i += kBlock) {
        double acc = 0.0;
        for (int j = 0; j < r; ++j) acc += (double)U[((int64_t)set * M.R + j) * M.n + i] * z[j];
        v[i] -= acc;
    }
}

void launch_smw_apply(const ModDev& M, int prec, double* V, int nrhs, int set0, int set_stride,
                      const int64_t* step_ptr, hipStream_t s)
{
    if (nrhs <= 0 || M.R <= 0) return;
    // one block per column: the endpoint gathers must see the unmodified v0
    if (prec == HINV_FP64)
        hipLaunchKernelGGL(k_smw_apply<double>, dim3(1, nrhs), dim3(kBlock), 0, s, M, (const double*)M.U, V, set0,
                           set_stride, step_ptr);
    else
        hipLaunchKernelGGL(k_smw_apply<float>, dim3(1, nrhs), dim3(kBlock), 0, s, M, (const float*)M.U32, V, set0,
                           set_stride, step_ptr);
}

// For every stored prefix r of set k: C_r = D_r^{-1} + W_r^T U_r (r x r, FP64),
// inverted by Gauss-Jordan with partial pivoting into Cinv slot r.  The
// changed G stays positive definite iff every new change's Schur complement
// 1 / Cinv_r[r-1][r-1] has the sign of its delta_g (Haynsworth inertia).
// Three-phase sets (M.grp3) change whole lines: D is block diagonal with the
// lines' 3x3 blocks, only prefixes ending on a line are formed (the three
// phases of a line become active together), and the new line keeps G positive
// definite iff its 3x3 block of Cinv_r (the inverse of its Schur complement)
// has the inertia of its D block, negative definite for a lost line.
__global__ void k_smw_capacitance(ModDev M, int* flags)
{
    const int set = blockIdx.x;
    if (threadIdx.x != 0) return;
    const int cnt = M.count[set];
    const int R = M.R;
    double A[kMaxModRank * kMaxModRank];
    double I[kMaxModRank * kMaxModRank];
    for (int r = 1; r <= cnt; ++r) {
        if (M.grp3 && r % 3 != 0) continue;
        for (int i = 0; i < r; ++i) {
            const int a = M.a[set * R + i], b = M.b[set * R + i];
            for (int j = 0; j < r; ++j) {
                const double* u = M.U + ((int64_t)set * R + j) * M.n;
                double v = u[a] - (b >= 0 ? u[b] : 0.0);
                if (M.grp3) {
                    if (i / 3 == j / 3) v += M.dinv3[((int64_t)set * R + i) * 3 + j % 3];
                } else if (i == j) {
                    v += 1.0 / M.dg[set * R + i];
                }
                A[i * r + j] = v;
                I[i * r + j] = (i == j) ? 1.0 : 0.0;
            }
        }
        bool ok = true;
        for (int k = 0; k < r && ok; ++k) {
            int p = k;
            for (int i = k + 1; i < r; ++i)
                if (fabs(A[i * r + k]) > fabs(A[p * r + k])) p = i;
            if (!(fabs(A[p * r + k]) > 0.0) || !isfinite(A[p * r + k])) { ok = false; break; }
            if (p != k)
                for (int j = 0; j < r; ++j) {
                    double t = A[k * r + j]; A[k * r + j] = A[p * r + j]; A[p * r + j] = t;
                    t = I[k * r + j]; I[k * r + j] = I[p * r + j]; I[p * r + j] = t;
                }
            const double piv = A[k * r + k];
            for (int j = 0; j < r; ++j) { A[k * r + j] /= piv; I[k * r + j] /= piv; }
            for (int i = 0; i < r; ++i) {
                if (i == k) continue;
                const double f = A[i * r + k];
                if (f == 0.0) continue;
                for (int j = 0; j < r; ++j) { A[i * r + j] -= f * A[k * r + j]; I[i * r + j] -= f * I[k * r + j]; }
            }
        }
        double* out = M.Cinv + ((int64_t)set * R + (r - 1)) * R * R;
        if (!ok) { atomicOr(flags, kFlagSingular); return; }
        for (int i = 0; i < r; ++i)
            for (int j = 0; j < r; ++j) out[i * R + j] = I[i * r + j];
        if (M.grp3) {           // -block SPD by its leading minors (a lost line: D negative definite)
            const double* B = I + (r - 3) * r + (r - 3);
            const double m1 = -B[0];
            const double m2 = B[0] * B[r + 1] - B[1] * B[r];
            const double m3 = -(B[0] * (B[r + 1] * B[2 * r + 2] - B[r + 2] * B[2 * r + 1]) -
                                B[1] * (B[r] * B[2 * r + 2] - B[r + 2] * B[2 * r]) +
                                B[2] * (B[r] * B[2 * r + 1] - B[r + 1] * B[2 * r]));
            if (!(m1 > 0.0 && m2 > 0.0 && m3 > 0.0)) atomicOr(flags, kFlagNotSPD);
            continue;
        }
        const double schur_inv = I[(r - 1) * r + (r - 1)];
        if (!((schur_inv > 0.0) == (M.dg[set * R + r - 1] > 0.0))) atomicOr(flags, kFlagNotSPD);
    }
}

void launch_smw_capacitance(const ModDev& M, int* flags, hipStream_t s)
{
    if (M.n_sets > 0 && M.R > 0) hipLaunchKernelGGL(k_smw_capacitance, dim3(M.n_sets), dim3(64), 0, s, M, flags);
}

// r = b - G_step v, column k uses change set k.
__global__ __launch_bounds__(kBlock) void k_residual(HierDev H, ModDev M, const double* __restrict__ Bv,
                                                      const double* __restrict__ V, double* __restrict__ Rv,
                                                      int set_stride, const int64_t* step_ptr)
{
    const int k = blockIdx.y, set = k * set_stride;
    const int64_t c = (int64_t)k * H.n;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= H.n) return;
    double acc = 0.0;
    for (int e = H.rp[i]; e < H.rp[i + 1]; ++e) acc += H.cv[e] * V[c + H.ci[e]];
    if (M.R > 0) {
        const int r = active_count(M, set, step_ptr);
        for (int j = 0; j < r; ++j) {
            const int a = M.a[set * M.R + j], b = M.b[set * M.R + j];
            if (i != a && i != b) continue;
            if (M.grp3) {          // row j of the line's 3x3 D times its three phase differences
                const int g0 = j - j % 3;
                const double* d = M.d3 + ((int64_t)set * M.R + j) * 3;
                double dw = 0.0;
                for (int q = 0; q < 3; ++q) {
                    const int aq = M.a[set * M.R + g0 + q], bq = M.b[set * M.R + g0 + q];
                    dw += d[q] * (V[c + aq] - (bq >= 0 ? V[c + bq] : 0.0));
                }
                acc += (i == a ? 1.0 : -1.0) * dw;
                continue;
            }
            const double wv = V[c + a] - (b >= 0 ? V[c + b] : 0.0);
            acc += (i == a ? 1.0 : -1.0) * M.dg[set * M.R + j] * wv;
        }
    }
    Rv[c + i] = Bv[c + i] - acc;
}

void launch_residual(const HierDev& H, const ModDev& M, const double* Bv, const double* V, double* Rv, int nrhs,
                     int set_stride, const int64_t* step_ptr, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual, dim3((H.n + kBlock - 1) / kBlock, nrhs), dim3(kBlock), 0, s, H, M, Bv, V, Rv,
                       set_stride, step_ptr);
}

__device__ inline void atomic_max_nonneg(unsigned long long* p, double v)
{
    atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// v += d for one column per block; the column's max|d| / max|v| is folded
// into stats[k] (max over calls) and flags kFlagNoConv when above rel_tol.
__global__ __launch_bounds__(kBlock) void k_axpy_stats(int n, double* __restrict__ V, const double* __restrict__ D,
                                                        unsigned long long* stats, double rel_tol, int* flags)
{
    __shared__ double md[kBlock], mv[kBlock];
    const int k = blockIdx.y;
    const int64_t c = (int64_t)k * n;
    double dmax = 0.0, vmax = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) {
        const double d = D[c + i];
        const double v = V[c + i] + d;
        V[c + i] = v;
        dmax = fmax(dmax, fabs(d));
        vmax = fmax(vmax, fabs(v));
    }
    if (!stats) return;
    md[threadIdx.x] = dmax;
    mv[threadIdx.x] = vmax;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            md[threadIdx.x] = fmax(md[threadIdx.x], md[threadIdx.x + off]);
            mv[threadIdx.x] = fmax(mv[threadIdx.x], mv[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ratio = mv[0] > 0.0 ? md[0] / mv[0] : (md[0] > 0.0 ? INFINITY : 0.0);
        if (!isfinite(ratio)) {
            atomicOr(flags, kFlagNaN);
        } else {
            atomic_max_nonneg(&stats[k], ratio);
            if (ratio > rel_tol) atomicOr(flags, kFlagNoConv);
        }
    }
}

void launch_axpy_stats(int n, int nrhs, double* V, const double* D, unsigned long long* stats, double rel_tol,
                       int* flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy_stats, dim3(1, nrhs), dim3(kBlock), 0, s, n, V, D, stats, rel_tol, flags);
}

}  // namespace hinv
