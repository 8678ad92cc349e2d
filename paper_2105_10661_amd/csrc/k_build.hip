// FP64 build of the exact hierarchical inverse on the GPU (Algorithm 1 of the
// paper, Section III.B, with the coupling level made exact).
//
//  leaf_inverse : B_l^{-1} of every leaf block (principal submatrix of G), by
//                 Gauss-Jordan elimination in registers, one workgroup per leaf.
//                 G is SPD, so every leaf block is SPD and needs no pivoting; a
//                 pivot <= 0 means the input was not SPD and is flagged.
//  build_z      : column j of Z_t = w_j G_c^{-1} e_a, where a is the line
//                 endpoint in child c.  Computed from the already built lower
//                 levels: the leaf inverse column, then the Woodbury update of
//                 every ancestor of the leaf below t (the vector stays inside
//                 the ancestor's rows, so only that ancestor's level is needed).
//                 This is the paper's G_l^{-1} h_l of Eq. (9).
//  node_inverse : S_t = C_t + U_t^T Z_t assembled and inverted (Gauss-Jordan
//                 with partial pivoting: S is symmetric but indefinite) in
//                 registers, one workgroup per node of order <= 128.
//  fill_s, gj_* : the same for larger nodes: S^T written into the S^{-1} slot
//                 (Gauss-Jordan on S^T yields S^{-1} column-major), then
//                 in-place elimination for all listed nodes at once, one launch
//                 pair per pivot step.
#include "hinv_internal.h"
#include "team_sync.h"

namespace hinv {

// Every builder takes an optional list of the leaves / columns / nodes to (re)build (NULL: all of
// them, or all of the level); a local line update rebuilds only what the change reaches.

// Register-resident Gauss-Jordan inversion of one matrix of order m <= kGjMax per workgroup of
// kGjThreads threads.  Thread (ti, tj) = (tid / 32, tid % 32) holds the entries (ti + 32a, tj + 32b),
// a, b < 4, so a pivot step moves only the pivot column and the scaled pivot row through LDS
// (double-buffered by step parity).  No rows are swapped: with partial pivoting (gj_regs, three
// barriers per step), step k takes the unused row r_k of largest |x[r][k]|, and at the end entry
// (i, j) of the eliminated matrix is entry (s_i, r_j) of the inverse, s = r^{-1}.  SPD leaf blocks,
// whose diagonal pivots stay positive, take r_k = k (gj_chunk_spd, two barriers per step).
constexpr int kGjThreads = 1024;
constexpr int kGjMax = kNodeGjMax;
static_assert(kMaxLeaf <= kGjMax, "leaf blocks are inverted by the register-resident kernel");

struct GjShared {
    double colk[2][kGjMax];
    double rowr[2][kGjMax];
    int rk[kGjMax];
    int sk[kGjMax];
    int used[kGjMax];
};

__device__ bool gj_regs(double (&x)[4][4], int m, GjShared& sh)
{
    const int tid = threadIdx.x, ti = tid >> 5, tj = tid & 31;
    for (int i = tid; i < m; i += kGjThreads) sh.used[i] = 0;
    for (int k = 0; k < m; ++k) {
        double* ck = sh.colk[k & 1];
        double* rr = sh.rowr[k & 1];
        if (tj == (k & 31)) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (b == (k >> 5)) {
#pragma unroll
                    for (int a = 0; a < 4; ++a)
                        if (ti + 32 * a < m) ck[ti + 32 * a] = x[a][b];
                }
        }
        __syncthreads();
        {
            if (tid < 64) {
                double bv = -1.0;
                int bi = m;
                for (int i = tid; i < m; i += 64) {
                    const double v = fabs(ck[i]);
                    if (!sh.used[i] && v > bv) { bv = v; bi = i; }
                }
                for (int off = 32; off > 0; off >>= 1) {
                    const double ov = __shfl_xor(bv, off);
                    const int oi = __shfl_xor(bi, off);
                    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
                }
                if (tid == 0) {
                    sh.rk[k] = bi;             // m: no usable row left (NaN column)
                    if (bi < m) { sh.sk[bi] = k; sh.used[bi] = 1; }
                }
            }
            __syncthreads();
            if (sh.rk[k] >= m) return false;   // uniform
        }
        const int r = sh.rk[k];
        const double p = ck[r];
        if (!(fabs(p) > 0.0) || !isfinite(p)) return false;   // uniform
        if (ti == (r & 31)) {
            const double pinv = 1.0 / p;
#pragma unroll
            for (int a = 0; a < 4; ++a)
                if (a == (r >> 5)) {
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int j = tj + 32 * b;
                        if (j < m) rr[j] = (j == k) ? pinv : x[a][b] * pinv;
                    }
                }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int i = ti + 32 * a;
            if (i >= m) continue;
            const double f = ck[i];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = tj + 32 * b;
                if (j >= m) continue;
                if (i == r) x[a][b] = rr[j];
                else if (j == k) x[a][b] = -f * rr[k];
                else x[a][b] -= f * rr[j];
            }
        }
    }
    return true;
}

// The pivot-free form for SPD blocks (r_k = k), as four chunks of 32 steps so that the tile row /
// column holding pivot k is a compile-time index: the pivot column and the scaled pivot row go
// through LDS, and the update x[i][j] <- x[i][j] - x[i][k] rr[j] takes the pivot row (i = k:
// x = rr[j]) and the pivot column (j = k: x = -x[i][k] / p) by zeroing the base term.
template <int KB>
__device__ __forceinline__ bool gj_chunk_spd(double (&x)[4][4], int m, GjShared& sh)
{
    const int tid = threadIdx.x, ti = tid >> 5, tj = tid & 31;
    for (int kk = 0; kk < 32; ++kk) {
        const int k = KB * 32 + kk;
        if (k >= m) return true;
        double* ck = sh.colk[k & 1];
        double* rr = sh.rowr[k & 1];
        if (tj == kk) {
#pragma unroll
            for (int a = 0; a < 4; ++a) ck[ti + 32 * a] = x[a][KB];
        }
        __syncthreads();
        const double p = ck[k];
        if (!(p > 0.0) || !isfinite(p)) return false;      // uniform
        const double pinv = 1.0 / p;
        if (ti == kk) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = tj + 32 * b;
                rr[j] = (j == k) ? pinv : x[KB][b] * pinv;
            }
        }
        __syncthreads();
        double rj[4], fa[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) rj[b] = rr[tj + 32 * b];
#pragma unroll
        for (int a = 0; a < 4; ++a) fa[a] = ck[ti + 32 * a];
        const bool prow = (ti == kk), pcol = (tj == kk);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const double f = (a == KB && prow) ? -1.0 : fa[a];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                double base = x[a][b];
                if (a == KB) base = prow ? 0.0 : base;
                if (b == KB) base = pcol ? 0.0 : base;
                x[a][b] = base - f * rj[b];
            }
        }
    }
    return true;
}

// B_l^{-1} of each listed leaf block (principal submatrix of G), written column-major.  The
// block is assembled in LDS from the leaf's contiguous CSR range (coalesced loads), then moved to
// registers.  A pivot <= 0 means G is not SPD and is flagged.
__global__ __launch_bounds__(kGjThreads) void k_leaf_inverse(HierDev H, int* flags, const int* list)
{
    __shared__ GjShared sh;
    __shared__ double A[kMaxLeaf * kMaxLeaf];
    __shared__ int rps[kMaxLeaf + 1];
    const int l = list ? list[blockIdx.x] : (int)blockIdx.x;
    const int lo = H.leaf_lo[l], nl = H.leaf_n[l];
    const int tid = threadIdx.x, ti = tid >> 5, tj = tid & 31;
    for (int idx = tid; idx < nl * nl; idx += kGjThreads) A[idx] = 0.0;
    for (int i = tid; i <= nl; i += kGjThreads) rps[i] = H.rp[lo + i];
    __syncthreads();
    const int e0 = rps[0], e1 = rps[nl];
    for (int e = e0 + tid; e < e1; e += kGjThreads) {
        const int c = H.ci[e] - lo;
        if (c < 0 || c >= nl) continue;
        int r0 = 0, r1 = nl;                 // row: rps[r] <= e < rps[r + 1]
        while (r1 - r0 > 1) {
            const int mid = (r0 + r1) >> 1;
            if (rps[mid] <= e) r0 = mid; else r1 = mid;
        }
        A[r0 * nl + c] = H.cv[e];
    }
    __syncthreads();
    double x[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ti + 32 * a, j = tj + 32 * b;
            x[a][b] = (i < nl && j < nl) ? A[i * nl + j] : 0.0;
        }
    const bool ok = gj_chunk_spd<0>(x, nl, sh) && gj_chunk_spd<1>(x, nl, sh) && gj_chunk_spd<2>(x, nl, sh) &&
                    gj_chunk_spd<3>(x, nl, sh);
    if (!ok) {
        if (tid == 0) atomicOr(flags, kFlagNotSPD);
        return;
    }
    double* out = H.blk + H.leaf_off[l];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ti + 32 * a, j = tj + 32 * b;
            if (i < nl && j < nl) out[(int64_t)j * nl + i] = x[a][b];
        }
}

// S_t^{-1} of each listed node with m <= kGjMax: S = C + U^T Z assembled in registers (transposed,
// as the S^{-1} slot holds S^{-1} column-major; the column data staged in LDS first), inverted
// with partial pivoting.
__global__ __launch_bounds__(kGjThreads) void k_node_inverse(HierDev H, const int* list, int* flags)
{
    __shared__ GjShared sh;
    __shared__ int cpart[kGjMax], crow[kGjMax], cplo[kGjMax], cpn[kGjMax];
    __shared__ double csg[kGjMax], cw[kGjMax];
    __shared__ int64_t czo[kGjMax];
    const int t = list[blockIdx.x];
    const int m = H.node_m[t], c0 = H.node_col0[t];
    const int tid = threadIdx.x, ti = tid >> 5, tj = tid & 31;
    if (tid < m) {
        const int g = c0 + tid;
        const int P = H.col_pan[g];
        cpart[tid] = H.col_partner[g] - c0;
        csg[tid] = H.col_sign[g];
        crow[tid] = H.col_row[g];
        cw[tid] = H.col_w[g];
        cplo[tid] = H.pan_lo[P];
        cpn[tid] = H.pan_n[P];
        czo[tid] = H.pan_zoff[P] + (int64_t)(g - H.pan_col0[P]) * H.pan_n[P];
    }
    __syncthreads();
    double x[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ti + 32 * a, j = tj + 32 * b;     // x[i][j] = S[j][i]: p = j, q = i
            double v = 0.0;
            if (i < m && j < m) {
                if (cpart[j] == i) v = csg[j];
                const int rp = crow[j] - cplo[i];
                if (rp >= 0 && rp < cpn[i]) v += cw[j] * H.Z[czo[i] + rp];
            }
            x[a][b] = v;
        }
    if (!gj_regs(x, m, sh)) {
        if (tid == 0) atomicOr(flags, kFlagSingular);
        return;
    }
    double* out = H.Sinv + H.node_soff[t];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ti + 32 * a, j = tj + 32 * b;
            if (i < m && j < m) out[(int64_t)sh.sk[i] * m + sh.rk[j]] = x[a][b];
        }
}

// S_t^{-1} of each listed node of order kNodeGjMax < m <= kGjTeamMax, by a team of ceil(m / 16)
// workgroups per node (one cooperative launch for all listed nodes).  Workgroup w holds the
// 16-column slice [16w, 16w + 16) of the matrix (S^T, assembled in place), one row per thread in
// registers.  Panel q: its owner runs the 16 pivot steps of columns 16q.. on its own slice, publishes
// the eliminated slice and its pivot rows P, and after one team barrier every other workgroup
// applies the whole panel at once to its slice J: rows of P become T A[P, J] and the others
// A[i, J] + X[i, K] A[P, J], with T = A[P, K]^{-1} and X[i, K] = -A[i, K] T as the owner left them
// (block Gauss-Jordan: the same result as sixteen single steps).  One team barrier per 16 pivots;
// the exchange goes through the device-scope accessors of the team barrier.
//
// A pivot step takes one workgroup barrier: every thread whose row is not yet a pivot keeps a copy
// of its row in LDS, the pivot is chosen by a wave-level maximum of 32-bit keys (the high word of
// |x| with its low 10 bits replaced by 1023 - row: the largest |x| up to a relative 2^-10, ties to
// the lowest row; partial pivoting needs no more) and each thread reads the pivot row's copy; the
// pivot row's thread stops updating its copy from then on, so no copy that is being read is
// written.  No rows are swapped; at the end entry (i, j) is entry (s_i, r_j) of the inverse.  A
// pivot that is zero or not finite raises kFlagSingular; the whole team stops after the same
// barrier.
constexpr int kGjNB = 16;
constexpr int kGjMS = kGjNB + 1;    // row stride of the LDS row copies: 17 doubles, so the rows of a
                                    // wavefront's lanes start in different banks (16 put them all in one)
constexpr int kGjTeamThreads = 1024;
static_assert(kGjTeamMax <= kGjTeamThreads, "one row per thread");

struct GjTeamLayout {
    size_t mir, oldp, wmax, rof, sof, piv, ctl, cpart, crow, csg, cw, total;
};

__host__ __device__ inline GjTeamLayout gj_team_layout(int mmax)
{
    GjTeamLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = (off + bytes + 15) / 16 * 16; return o; };
    L.mir = take(sizeof(double) * (size_t)mmax * kGjMS);     // row i's copy at i * kGjMS
    L.oldp = take(sizeof(double) * kGjNB * kGjNB);
    L.wmax = take(sizeof(unsigned) * 32);
    L.rof = take(sizeof(int) * (size_t)mmax);
    L.sof = take(sizeof(int) * (size_t)mmax);
    L.piv = take(sizeof(int) * kGjNB);
    L.ctl = take(sizeof(int) * 4);
    L.cpart = take(sizeof(int) * kGjNB);
    L.crow = take(sizeof(int) * kGjNB);
    L.csg = take(sizeof(double) * kGjNB);
    L.cw = take(sizeof(double) * kGjNB);
    L.total = off;
    return L;
}

// Maximum over the wavefront (all 64 lanes active): rotations within rows of 16, then the four rows.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v)
{
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false));   // row_ror:8
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false));   // row_ror:4
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x122, 0xF, 0xF, false));   // row_ror:2
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x121, 0xF, 0xF, false));   // row_ror:1
    const unsigned a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    const unsigned c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return max(max(a, b), max(c, d));
}

struct GjTeamStep {
    double* mir;
    unsigned* wmax;
    int* rof;
    int* sof;
    int k0, tid, lane, wave;
};

// Pivot step KK of the owner's panel (column k0 + KK of the matrix, column KK of the slice).
template <int KK>
__device__ __forceinline__ void gj_team_step(double (&x)[kGjNB], int& used, bool& bad, const GjTeamStep& S)
{
    const double xk = x[KK];
    unsigned key = 0;
    if (!used) {
        const double a = fabs(xk);
        if (a == a) key = ((unsigned)(__double_as_longlong(a) >> 32) & ~0x3FFu) | (1023u - (unsigned)S.tid);
    }
    key = wave_max_u32(key);
    if (S.lane == 0) S.wmax[(KK & 1) * 16 + S.wave] = key;
    __syncthreads();
    unsigned kv = 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) kv = max(kv, S.wmax[(KK & 1) * 16 + v]);   // unused slots hold 0
    if (kv == 0) { bad = true; return; }                                      // uniform
    const int r = 1023 - (int)(kv & 0x3FF);
    double pr[kGjNB];
#pragma unroll
    for (int jj = 0; jj < kGjNB; ++jj) pr[jj] = S.mir[r * kGjMS + jj];
    const double p = pr[KK];
    if (!(fabs(p) > 0.0) || !isfinite(p)) { bad = true; return; }
    const double pinv = 1.0 / p;
#pragma unroll
    for (int jj = 0; jj < kGjNB; ++jj) pr[jj] = (jj == KK) ? pinv : pr[jj] * pinv;
    if (S.tid == 0) { S.rof[S.k0 + KK] = r; S.sof[r] = S.k0 + KK; }
    if (S.tid == r) {
        used = 1;
#pragma unroll
        for (int jj = 0; jj < kGjNB; ++jj) x[jj] = pr[jj];
    } else {
#pragma unroll
        for (int jj = 0; jj < kGjNB; ++jj) x[jj] = (jj == KK) ? -xk * pinv : x[jj] - xk * pr[jj];
        if (!used)
#pragma unroll
            for (int jj = 0; jj < kGjNB; ++jj) S.mir[S.tid * kGjMS + jj] = x[jj];
    }
}

__global__ __launch_bounds__(kGjTeamThreads) void k_gj_team(HierDev H, const int* list, int count, int mmax,
                                                           double* xb, unsigned int* sync, int* flags)
{
    extern __shared__ __align__(16) unsigned char gj_lds[];
    const GjTeamLayout L = gj_team_layout(mmax);
    double* mir = (double*)(gj_lds + L.mir);
    double* oldp = (double*)(gj_lds + L.oldp);
    unsigned* wmax = (unsigned*)(gj_lds + L.wmax);
    int* rof = (int*)(gj_lds + L.rof);
    int* sof = (int*)(gj_lds + L.sof);
    int* piv = (int*)(gj_lds + L.piv);
    int* ctl = (int*)(gj_lds + L.ctl);
    int* cpart = (int*)(gj_lds + L.cpart);
    int* crow = (int*)(gj_lds + L.crow);
    double* csg = (double*)(gj_lds + L.csg);
    double* cw = (double*)(gj_lds + L.cw);
    // this workgroup's node and slice
    int acc = 0, t = -1, m = 0, W = 0;
    int64_t xoff = 0;
    for (int n = 0; n < count; ++n) {
        t = list[n];
        m = H.node_m[t];
        W = (m + kGjNB - 1) / kGjNB;
        if ((int)blockIdx.x < acc + W) break;
        acc += W;
        xoff += 2 * ((int64_t)m * kGjNB + kGjNB);
    }
    const int w = (int)blockIdx.x - acc;
    unsigned int* flg = sync + acc;
    const int c0 = H.node_col0[t];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j0 = w * kGjNB, nw = min(kGjNB, m - j0);
    const bool own = tid < m;
    if (tid < nw) {       // my columns in the role of p
        const int g = c0 + j0 + tid;
        cpart[tid] = H.col_partner[g] - c0;
        csg[tid] = H.col_sign[g];
        crow[tid] = H.col_row[g];
        cw[tid] = H.col_w[g];
    }
    if (tid < 32) wmax[tid] = 0u;
    __syncthreads();
    double x[kGjNB];
#pragma unroll
    for (int jj = 0; jj < kGjNB; ++jj) x[jj] = 0.0;
    if (own) {            // x[i][j] = S[j][i] = C[j][i] + w_j Z_i[row_j]
        const int g = c0 + tid;
        const int P = H.col_pan[g];
        const int plo = H.pan_lo[P], pn = H.pan_n[P];
        const double* zq = H.Z + H.pan_zoff[P] + (int64_t)(g - H.pan_col0[P]) * pn;
#pragma unroll
        for (int jj = 0; jj < kGjNB; ++jj) {
            if (jj < nw) {
                double v = (cpart[jj] == tid) ? csg[jj] : 0.0;
                const int rp = crow[jj] - plo;
                if (rp >= 0 && rp < pn) v += cw[jj] * zq[rp];
                x[jj] = v;
            }
        }
    }
    int used = own ? 0 : 1;
    unsigned int epoch = 0;
    for (int q = 0; q < W; ++q) {
        const int k0 = q * kGjNB, nk = min(kGjNB, m - k0);
        double* xq = xb + xoff + (int64_t)(q & 1) * ((int64_t)m * kGjNB + kGjNB);
        if (q == w) {
            if (!used)
#pragma unroll
                for (int jj = 0; jj < kGjNB; ++jj) mir[tid * kGjMS + jj] = x[jj];
            bool bad = false;
            const GjTeamStep S{mir, wmax, rof, sof, k0, tid, lane, wave};
#define HINV_GJ_STEP(K) if (K < nk && !bad) gj_team_step<K>(x, used, bad, S);
            HINV_GJ_STEP(0) HINV_GJ_STEP(1) HINV_GJ_STEP(2) HINV_GJ_STEP(3)
            HINV_GJ_STEP(4) HINV_GJ_STEP(5) HINV_GJ_STEP(6) HINV_GJ_STEP(7)
            HINV_GJ_STEP(8) HINV_GJ_STEP(9) HINV_GJ_STEP(10) HINV_GJ_STEP(11)
            HINV_GJ_STEP(12) HINV_GJ_STEP(13) HINV_GJ_STEP(14) HINV_GJ_STEP(15)
#undef HINV_GJ_STEP
            if (own && !bad)
#pragma unroll
                for (int jj = 0; jj < kGjNB; ++jj)
                    if (jj < nk) xchg_store(&xq[(int64_t)tid * kGjNB + jj], x[jj]);
            if (tid < kGjNB) xchg_store(&xq[(int64_t)m * kGjNB + tid], bad ? -1.0 : (tid < nk ? (double)rof[k0 + tid] : 0.0));
        }
        if (!team_barrier(flg, w, W, ++epoch, flags, ctl + 2)) return;
        double pv[kGjNB];    // the panel's transformed rows, loaded with the pivot list (one round trip)
#pragma unroll
        for (int b = 0; b < kGjNB; ++b) pv[b] = (own && q != w && b < nk) ? xchg_load(&xq[(int64_t)tid * kGjNB + b]) : 0.0;
        if (tid < kGjNB) piv[tid] = (int)xchg_load(&xq[(int64_t)m * kGjNB + tid]);
        __syncthreads();
        if (piv[0] < 0) {
            if (w == 0 && tid == 0) atomicOr(flags, kFlagSingular);
            return;                                                                   // whole team
        }
        if (q == w) continue;
        int mine = -1;    // this thread's row is pivot row mine of the panel
#pragma unroll
        for (int b = 0; b < kGjNB; ++b) mine = (b < nk && piv[b] == tid) ? b : mine;
        if (mine >= 0) {
#pragma unroll
            for (int jj = 0; jj < kGjNB; ++jj) oldp[mine * kGjNB + jj] = x[jj];
            used = 1;
        }
        if (tid < nk) { rof[k0 + tid] = piv[tid]; sof[piv[tid]] = k0 + tid; }
        __syncthreads();
        if (own) {
#pragma unroll
            for (int jj = 0; jj < kGjNB; ++jj) x[jj] = (mine >= 0) ? 0.0 : x[jj];
#pragma unroll
            for (int b = 0; b < kGjNB; ++b)
#pragma unroll
                for (int jj = 0; jj < kGjNB; ++jj) x[jj] += pv[b] * oldp[b * kGjNB + jj];
        }
        __syncthreads();
    }
    double* out = H.Sinv + H.node_soff[t];
    if (own)
#pragma unroll
        for (int jj = 0; jj < kGjNB; ++jj)
            if (jj < nw) out[(int64_t)sof[tid] * m + rof[j0 + jj]] = x[jj];
}

hipError_t launch_gj_team(const HierDev& H, const int* list, const std::vector<int>& m_of, double* xb,
                          unsigned int* sync, int* flags, hipStream_t s)
{
    if (m_of.empty()) return hipSuccess;
    const void* fn = (const void*)k_gj_team;
    const size_t lds_max = gj_team_layout(kGjTeamMax).total;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0, per = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kGjTeamThreads, lds_max)) != hipSuccess) return e;
    const int cap = per * cus;
    size_t i = 0;
    while (i < m_of.size()) {       // runs of nodes whose teams are resident at once
        int wgs = 0, mmax = 0;
        size_t j = i;
        while (j < m_of.size()) {
            const int W = (m_of[j] + kGjNB - 1) / kGjNB;
            if (j > i && wgs + W > cap) break;
            wgs += W;
            mmax = std::max(mmax, m_of[j]);
            ++j;
        }
        if (wgs > cap || mmax > kGjTeamMax) return hipErrorCooperativeLaunchTooLarge;
        if ((e = hipMemsetAsync(sync, 0, sizeof(unsigned int) * (size_t)wgs, s)) != hipSuccess) return e;
        HierDev Hc = H;
        const int* lst = list + i;
        int cnt = (int)(j - i);
        void* args[] = {&Hc, &lst, &cnt, &mmax, &xb, &sync, &flags};
        e = hipLaunchCooperativeKernel(fn, dim3(wgs), dim3((mmax + 63) / 64 * 64), args,
                                       (unsigned int)gj_team_layout(mmax).total, s);
        if (e != hipSuccess) return e;
        i = j;
    }
    return hipGetLastError();
}

// Exchange doubles and barrier flags launch_gj_team needs for nodes of these orders.
void gj_team_sizes(const std::vector<int>& m_of, int64_t* xb_doubles, int64_t* sync_words)
{
    int64_t x = 0, y = 0;
    for (int m : m_of) {
        x += 2 * ((int64_t)m * kGjNB + kGjNB);
        y += (m + kGjNB - 1) / kGjNB;
    }
    *xb_doubles = x;
    *sync_words = y;
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
// coupling_only: C alone (C^{-1} = C, the paper's approximation of S^{-1}).
// Grid (x: slices of the entries, y: listed nodes).
__global__ __launch_bounds__(kBlock) void k_fill_s(HierDev H, int level, const int* list, bool coupling_only)
{
    const int t = list ? list[blockIdx.y] : H.lvl_node[level - 1] + (int)blockIdx.y;
    const int m = H.node_m[t], c0 = H.node_col0[t];
    double* S = H.Sinv + H.node_soff[t];
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < m * m; idx += gridDim.x * blockDim.x) {
        const int q = idx / m, p = idx - q * m;
        const int gp = c0 + p, gq = c0 + q;
        double v = (H.col_partner[gp] == gq) ? H.col_sign[gp] : 0.0;
        const int P = H.col_pan[gq];
        const int rp = H.col_row[gp] - H.pan_lo[P];
        if (!coupling_only && rp >= 0 && rp < H.pan_n[P])
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
    if (nb > 0) hipLaunchKernelGGL(k_leaf_inverse, dim3(nb), dim3(kGjThreads), 0, s, H, flags, list);
}

void launch_build_z(const HierDev& H, int level, int ncols, hipStream_t s, const int* list)
{
    if (ncols <= 0) return;
    const size_t lds = sizeof(double) * 2 * (size_t)(H.max_cols > 0 ? H.max_cols : 1);
    hipLaunchKernelGGL(k_build_z, dim3(ncols), dim3(kBlock), lds, s, H, level, list);
}

void launch_fill_s(const HierDev& H, int level, int nnodes, int m_max, hipStream_t s, const int* list,
                   bool coupling_only)
{
    if (nnodes <= 0 || m_max <= 0) return;
    int gx = (int)(((int64_t)m_max * m_max + kBlock - 1) / kBlock);
    if (gx > 256) gx = 256;
    hipLaunchKernelGGL(k_fill_s, dim3(gx, nnodes), dim3(kBlock), 0, s, H, level, list, coupling_only);
}

void launch_node_inverse(const HierDev& H, const int* list, int count, int* flags, hipStream_t s)
{
    if (count > 0) hipLaunchKernelGGL(k_node_inverse, dim3(count), dim3(kGjThreads), 0, s, H, list, flags);
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
