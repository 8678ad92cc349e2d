// FP64 build of the exact hierarchical inverse on the GPU (Algorithm 1 of the
// paper, Section III.B, with the coupling level made exact).
//
//  leaf_inverse : B_l^{-1} of every leaf block (principal submatrix of G), by
//                 Gauss-Jordan elimination in LDS.  G is SPD, so every leaf
//                 block is SPD and needs no pivoting; a pivot <= 0 means the
//                 input was not SPD and is flagged.
//  build_z      : column j of Z_t = w_j G_c^{-1} e_a, where a is the line
//                 endpoint in child c.  Computed from the already built lower
//                 levels: the leaf inverse column, then the Woodbury update of
//                 every ancestor of the leaf below t (the vector stays inside
//                 the ancestor's rows, so only that ancestor's level is needed).
//                 This is the paper's G_l^{-1} h_l of Eq. (9).
//  fill_s       : S_t = C_t + U_t^T Z_t, written transposed into the S^{-1}
//                 slot (Gauss-Jordan on S^T yields S^{-1} column-major).
//  gj_*         : in-place Gauss-Jordan inversion with partial (row) pivoting
//                 for all nodes of a level at once, one launch pair per pivot
//                 step; S is symmetric but indefinite.
#include "hinv_internal.h"

namespace hinv {

// Every builder takes an optional list of the leaves / columns / nodes to (re)build (NULL: all of
// them, or all of the level); a local line update rebuilds only what the change reaches.
__global__ __launch_bounds__(kBlock) void k_leaf_inverse(HierDev H, int* flags, const int* list)
{
    __shared__ double A[kMaxLeaf * kMaxLeaf];
    __shared__ double rowk[kMaxLeaf];
    __shared__ double colk[kMaxLeaf];
    const int l = list ? list[blockIdx.x] : (int)blockIdx.x;
    const int lo = H.leaf_lo[l], nl = H.leaf_n[l];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < nl * nl; idx += blockDim.x) A[idx] = 0.0;
    __syncthreads();
    for (int i = tid; i < nl; i += blockDim.x) {
        const int r = lo + i;
        for (int e = H.rp[r]; e < H.rp[r + 1]; ++e) {
            const int c = H.ci[e] - lo;
            if (c >= 0 && c < nl) A[i * nl + c] = H.cv[e];
        }
    }
    __syncthreads();
    for (int k = 0; k < nl; ++k) {
        const double p = A[k * nl + k];
        if (!(p > 0.0) || !isfinite(p)) {      // uniform across the block
            if (tid == 0) atomicOr(flags, kFlagNotSPD);
            return;
        }
        for (int j = tid; j < nl; j += blockDim.x) rowk[j] = (j == k) ? 1.0 / p : A[k * nl + j] / p;
        for (int i = tid; i < nl; i += blockDim.x) colk[i] = A[i * nl + k];
        __syncthreads();
        for (int idx = tid; idx < nl * nl; idx += blockDim.x) {
            const int i = idx / nl, j = idx - i * nl;
            if (i == k) {
                A[idx] = rowk[j];
            } else {
                const double a = (j == k) ? 0.0 : A[idx];
                A[idx] = a - colk[i] * rowk[j];
            }
        }
        __syncthreads();
    }
    double* out = H.blk + H.leaf_off[l];
    for (int idx = tid; idx < nl * nl; idx += blockDim.x) {
        const int j = idx / nl, i = idx - j * nl;     // column-major out[j*nl+i] = inv[i][j]
        out[idx] = A[i * nl + j];
    }
}

// One block per coupling column of the level.
__global__ __launch_bounds__(kBlock) void k_build_z(HierDev H, int level, const int* list)
{
    extern __shared__ double sh[];
    double* s = sh;
    double* y = sh + H.max_cols;
    const int p = list ? list[blockIdx.x] : H.lvl_col[level - 1] + (int)blockIdx.x;
    const int P = H.col_pan[p];
    const int clo = H.pan_lo[P], cn = H.pan_n[P];
    double* z = H.Z + H.pan_zoff[P] + (int64_t)(p - H.pan_col0[P]) * cn;
    const int a = H.col_row[p];
    const double w = H.col_w[p];
    const int l = H.row_leaf[a];
    const int llo = H.leaf_lo[l], ln = H.leaf_n[l];
    const double* bcol = H.blk + H.leaf_off[l] + (int64_t)(a - llo) * ln;
    const int tid = threadIdx.x;
    for (int i = tid; i < cn; i += blockDim.x) {
        const int r = clo + i;
        z[i] = (r >= llo && r < llo + ln) ? w * bcol[r - llo] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < H.anc_stride; ++k) {
        const int t = H.leaf_anc[l * H.anc_stride + k];
        if (t < 0 || H.node_level[t] >= level) break;
        const int m = H.node_m[t], c0 = H.node_col0[t];
        for (int q = tid; q < m; q += blockDim.x) s[q] = H.col_w[c0 + q] * z[H.col_row[c0 + q] - clo];
        __syncthreads();
        const double* Si = H.Sinv + H.node_soff[t];
        for (int q = tid; q < m; q += blockDim.x) {
            double acc = 0.0;
            for (int j = 0; j < m; ++j) acc += Si[(int64_t)j * m + q] * s[j];
            y[q] = acc;
        }
        __syncthreads();
        const int pan0 = H.node_pan0[t], npan = H.node_npan[t];
        for (int pp = pan0; pp < pan0 + npan; ++pp) {
            const int plo = H.pan_lo[pp], pn = H.pan_n[pp], pm = H.pan_m[pp];
            const int yc = H.pan_col0[pp] - c0;
            const double* Zp = H.Z + H.pan_zoff[pp];
            for (int i = tid; i < pn; i += blockDim.x) {
                double acc = 0.0;
                for (int j = 0; j < pm; ++j) acc += Zp[(int64_t)j * pn + i] * y[yc + j];
                z[plo - clo + i] -= acc;
            }
        }
        __syncthreads();
    }
}

// S^T into the S^{-1} slot: slot[q*m + p] = S[p][q], S[p][q] = C[p][q] + w_p Z_q[row_p].
__global__ __launch_bounds__(kBlock) void k_fill_s(HierDev H, int level, const int* list)
{
    const int t = list ? list[blockIdx.x] : H.lvl_node[level - 1] + (int)blockIdx.x;
    const int m = H.node_m[t], c0 = H.node_col0[t];
    double* S = H.Sinv + H.node_soff[t];
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
        const int q = idx / m, p = idx - q * m;
        const int gp = c0 + p, gq = c0 + q;
        double v = (H.col_partner[gp] == gq) ? H.col_sign[gp] : 0.0;
        const int P = H.col_pan[gq];
        const int rp = H.col_row[gp] - H.pan_lo[P];
        if (rp >= 0 && rp < H.pan_n[P])
            v += H.col_w[gp] * H.Z[H.pan_zoff[P] + (int64_t)(gq - H.pan_col0[P]) * H.pan_n[P] + rp];
        S[idx] = v;
    }
}

// Pivot step k for every node of the level: choose the pivot row, swap, scale
// row k, save and clear column k of the other rows.
__global__ __launch_bounds__(kBlock) void k_gj_pivot(HierDev H, int level, int k, double* colbuf, int* ipiv,
                                                      int* flags, const int* list)
{
    __shared__ double bv[kBlock];
    __shared__ int bi[kBlock];
    const int t = list ? list[blockIdx.x] : H.lvl_node[level - 1] + (int)blockIdx.x;
    const int m = H.node_m[t];
    if (k >= m) return;
    double* A = H.Sinv + H.node_soff[t];
    double* cb = colbuf + H.node_col0[t];
    int* ip = ipiv + H.node_col0[t];
    const int tid = threadIdx.x;
    double best = -1.0;
    int bidx = k;
    for (int i = k + tid; i < m; i += blockDim.x) {
        const double v = fabs(A[(int64_t)i * m + k]);
        if (v > best) { best = v; bidx = i; }
    }
    bv[tid] = best;
    bi[tid] = bidx;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (tid < off) {
            const double o = bv[tid + off];
            const int oi = bi[tid + off];
            if (o > bv[tid] || (o == bv[tid] && oi < bi[tid])) { bv[tid] = o; bi[tid] = oi; }
        }
        __syncthreads();
    }
    const int pr = bi[0];
    const double pv = bv[0];
    if (!(pv > 0.0) || !isfinite(pv)) {
        if (tid == 0) { atomicOr(flags, kFlagSingular); ip[k] = k; }
        return;
    }
    if (tid == 0) ip[k] = pr;
    if (pr != k) {
        for (int j = tid; j < m; j += blockDim.x) {
            const double tmp = A[(int64_t)k * m + j];
            A[(int64_t)k * m + j] = A[(int64_t)pr * m + j];
            A[(int64_t)pr * m + j] = tmp;
        }
    }
    __syncthreads();
    const double pinv = 1.0 / A[(int64_t)k * m + k];
    __syncthreads();
    for (int j = tid; j < m; j += blockDim.x) {
        A[(int64_t)k * m + j] = (j == k) ? pinv : A[(int64_t)k * m + j] * pinv;
    }
    for (int i = tid; i < m; i += blockDim.x) {
        if (i == k) { cb[i] = 0.0; continue; }
        cb[i] = A[(int64_t)i * m + k];
        A[(int64_t)i * m + k] = 0.0;
    }
}

// Elimination for pivot step k: A[i][j] -= f_i * A[k][j], i != k.
__global__ __launch_bounds__(kBlock) void k_gj_eliminate(HierDev H, int level, int k, const double* colbuf,
                                                          const int* list)
{
    const int t = list ? list[blockIdx.y] : H.lvl_node[level - 1] + (int)blockIdx.y;
    const int m = H.node_m[t];
    if (k >= m) return;
    double* A = H.Sinv + H.node_soff[t];
    const double* cb = colbuf + H.node_col0[t];
    const int64_t total = (int64_t)m * m;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx / m), j = (int)(idx - (int64_t)i * m);
        if (i == k) continue;
        A[idx] -= cb[i] * A[(int64_t)k * m + j];
    }
}

// Undo the row interchanges: swap columns k and ipiv[k], k from last to first.
__global__ __launch_bounds__(kBlock) void k_gj_unscramble(HierDev H, int level, const int* ipiv, const int* list)
{
    const int t = list ? list[blockIdx.x] : H.lvl_node[level - 1] + (int)blockIdx.x;
    const int m = H.node_m[t];
    double* A = H.Sinv + H.node_soff[t];
    const int* ip = ipiv + H.node_col0[t];
    for (int k = m - 1; k >= 0; --k) {
        const int p = ip[k];
        if (p != k) {
            for (int i = threadIdx.x; i < m; i += blockDim.x) {
                const double tmp = A[(int64_t)i * m + k];
                A[(int64_t)i * m + k] = A[(int64_t)i * m + p];
                A[(int64_t)i * m + p] = tmp;
            }
        }
        __syncthreads();
    }
}

__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

// FP64 -> BF16, round to nearest even (through FP32; NaN stays NaN).
__device__ inline uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ void k_to_bf16(const double* __restrict__ src, uint16_t* __restrict__ dst, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = f32_to_bf16((float)src[i]);
}

// float -> OCP E4M3 (round to nearest even, saturating at +-448).
__device__ inline uint8_t f32_to_e4m3(float f)
{
    const uint8_t sgn = f < 0.0f ? 0x80 : 0;
    float a = fabsf(f);
    if (!(a > 0.0f)) return sgn;
    if (a >= 448.0f) return sgn | 0x7e;                       // 1.75 * 2^8
    int e;
    frexpf(a, &e);                                            // a = f * 2^e, f in [0.5, 1)
    int eu = e - 1;                                           // a in [2^eu, 2^(eu+1))
    if (eu < -6) {                                            // subnormal: units of 2^-9
        const float q = rintf(ldexpf(a, 9));
        const int m = (int)q;
        return sgn | (uint8_t)(m >= 8 ? (1 << 3) : m);
    }
    int m = (int)rintf((ldexpf(a, -eu) - 1.0f) * 8.0f);
    if (m == 8) { m = 0; ++eu; }
    if (eu > 8 || (eu == 8 && m > 6)) return sgn | 0x7e;
    return sgn | (uint8_t)(((eu + 7) << 3) | m);
}

// One block per 32-entry group: scale 2^k, smallest k with max|x| / 2^k <= 448.
__global__ void k_to_fp8(const double* __restrict__ src, uint8_t* __restrict__ dst, uint8_t* __restrict__ scale,
                         int64_t count)
{
    const int64_t groups = (count + 31) / 32;
    const int lane = threadIdx.x & 31;
    for (int64_t gi = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 32; gi < groups;
         gi += ((int64_t)gridDim.x * blockDim.x) / 32) {
        const int64_t i = gi * 32 + lane;
        const float x = i < count ? (float)src[i] : 0.0f;
        float amax = fabsf(x);
        for (int o = 16; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 32));
        int k = 0;
        if (amax > 0.0f) {
            int e;
            frexpf(amax / 448.0f, &e);                        // amax/448 in [2^(e-1), 2^e)
            k = e;
            if (ldexpf(amax, -(k - 1)) <= 448.0f) k = k - 1;
        }
        k = k < -127 ? -127 : (k > 127 ? 127 : k);
        if (lane == 0) scale[gi] = (uint8_t)(k + 127);
        if (i < count) dst[i] = f32_to_e4m3(ldexpf(x, -k));
    }
}

void launch_to_bf16(const double* src, uint16_t* dst, int64_t count, hipStream_t s)
{
    if (count <= 0) return;
    int64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)blocks), dim3(kBlock), 0, s, src, dst, count);
}

void launch_to_fp8(const double* src, uint8_t* dst, uint8_t* scale, int64_t count, hipStream_t s)
{
    if (count <= 0) return;
    int64_t blocks = ((count + 31) / 32 * 32 + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_to_fp8, dim3((unsigned)blocks), dim3(kBlock), 0, s, src, dst, scale, count);
}

void launch_leaf_inverse(const HierDev& H, int* flags, hipStream_t s, const int* list, int count)
{
    const int nb = list ? count : H.n_leaves;
    if (nb > 0) hipLaunchKernelGGL(k_leaf_inverse, dim3(nb), dim3(kBlock), 0, s, H, flags, list);
}

void launch_build_z(const HierDev& H, int level, int ncols, hipStream_t s, const int* list)
{
    if (ncols <= 0) return;
    const size_t lds = sizeof(double) * 2 * (size_t)(H.max_cols > 0 ? H.max_cols : 1);
    hipLaunchKernelGGL(k_build_z, dim3(ncols), dim3(kBlock), lds, s, H, level, list);
}

void launch_fill_s(const HierDev& H, int level, int nnodes, hipStream_t s, const int* list)
{
    if (nnodes > 0) hipLaunchKernelGGL(k_fill_s, dim3(nnodes), dim3(kBlock), 0, s, H, level, list);
}

void launch_to_f32(const double* src, float* dst, int64_t count, hipStream_t s)
{
    if (count <= 0) return;
    int64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)blocks), dim3(kBlock), 0, s, src, dst, count);
}

// Gauss-Jordan of all capacitance matrices of one level (m_max: largest m of
// the level).  colbuf [n_cols] doubles and ipiv [n_cols] ints, indexed by the
// node's first global column.
void launch_gj_level(const HierDev& H, int level, int nnodes, int m_max, double* colbuf, int* ipiv, int* flags,
                     hipStream_t s, const int* list)
{
    if (nnodes <= 0 || m_max <= 0) return;
    const int64_t tot = (int64_t)m_max * m_max;
    int gx = (int)((tot + kBlock - 1) / kBlock);
    if (gx > 1024) gx = 1024;
    for (int k = 0; k < m_max; ++k) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(nnodes), dim3(kBlock), 0, s, H, level, k, colbuf, ipiv, flags, list);
        hipLaunchKernelGGL(k_gj_eliminate, dim3(gx, nnodes), dim3(kBlock), 0, s, H, level, k, colbuf, list);
    }
    hipLaunchKernelGGL(k_gj_unscramble, dim3(nnodes), dim3(kBlock), 0, s, H, level, ipiv, list);
}

}  // namespace hinv
