// Krylov kernels of the GMRES-based refinement (hinv_solve_gmres): the network equation G v = i of
// Section II, Eq. (2), solved to FP64 accuracy with the stored inverse applied in a low storage
// precision as a right preconditioner P.  The outer loop is iterative refinement in FP64 (residual
// r = b - G x with the sparse G); each correction solves G d = r by flexible GMRES on G P:
//   v_0 = r / ||r||;  for j: z_j = P v_j,  w = G z_j,  w <- w - sum_i h_ij v_i (classical
//   Gram-Schmidt, applied twice), h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j};
//   the small least-squares problem min || beta e_1 - H y || is kept triangular by Givens rotations,
//   its residual |g_{j+1}| tracked per column, and d = sum_j y_j z_j at the end.
// The preconditioner may be followed by damped-Jacobi sweeps z += (2/3) D^{-1} (v - G z): the error
// of a coarsely stored inverse is spread over all frequencies and G amplifies its high-frequency part
// most, which is what a Jacobi sweep damps (P alone is then a coarse correction and the sweeps its
// smoother; the composite is still one fixed linear operator, so GMRES on G M applies as before).
// All vectors are FP64 in the hierarchy's row order, nrhs columns side by side; each column runs its
// own Krylov space.  The host computes w as the residual kernel's 0 - G z (so every sign below that
// touches w carries that minus).  Small per-column arrays live in global memory and are handled by
// one thread per column.
#include "hinv_internal.h"

namespace hinv {

namespace {

constexpr int kGThreads = 256;

__device__ inline double block_sum(double x, double* red)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = x;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kGThreads / 64; ++q) s += red[q];
    return s;
}

// out[k * ld_out + i] = sgn * <V_i,k , W_k> for i = 0..nv-1 (one workgroup per (i, k)); with
// sqrt_out, sqrt of it (V = W, nv = 1: the column norms).
__global__ __launch_bounds__(kGThreads) void k_gm_dots(int n, int nrhs, const double* __restrict__ V,
                                                       const double* __restrict__ W, double sgn,
                                                       double* __restrict__ out, int ld_out, int sqrt_out)
{
    __shared__ double red[kGThreads / 64];
    const int i = blockIdx.x, k = blockIdx.y;
    const double* v = V + ((int64_t)i * nrhs + k) * n;
    const double* w = W + (int64_t)k * n;
    double acc = 0.0;
    for (int r = threadIdx.x; r < n; r += kGThreads) acc = fma(v[r], w[r], acc);
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[(int64_t)k * ld_out + i] = sqrt_out ? sqrt(s) : sgn * s;
}

// W_k += sgn * sum_{i < nv} h[k * ld_h + i] V_i,k
__global__ __launch_bounds__(kGThreads) void k_gm_update(int n, int nrhs, int nv, const double* __restrict__ V,
                                                         const double* __restrict__ h, int ld_h, double sgn,
                                                         double* __restrict__ W)
{
    const int k = blockIdx.y;
    const int r = blockIdx.x * kGThreads + threadIdx.x;
    if (r >= n) return;
    double acc = 0.0;
    for (int i = 0; i < nv; ++i) acc = fma(h[(int64_t)k * ld_h + i], V[((int64_t)i * nrhs + k) * n + r], acc);
    W[(int64_t)k * n + r] += sgn * acc;
}

// Vout_k = sgn * W_k / nrm[k] (zero when the column's norm is zero: its Krylov space is exhausted).
__global__ __launch_bounds__(kGThreads) void k_gm_scale(int n, const double* __restrict__ W,
                                                        const double* __restrict__ nrm, int ld_nrm, double sgn,
                                                        double* __restrict__ Vout)
{
    const int k = blockIdx.y;
    const int r = blockIdx.x * kGThreads + threadIdx.x;
    if (r >= n) return;
    const double s = nrm[(int64_t)k * ld_nrm];
    Vout[(int64_t)k * n + r] = s > 0.0 ? sgn * W[(int64_t)k * n + r] / s : 0.0;
}

// Column j of each column's Hessenberg matrix: h_ij = h1_ij + h2_ij (the two Gram-Schmidt passes),
// h_{j+1,j} = ||w||; the previous rotations applied to it, a new rotation zeroing h_{j+1,j}, and the
// rotated right-hand side g.  res[k] = |g_{j+1}|, the column's GMRES residual norm.
// Layout per column k: Hs[k][(m+1) * m] column-major (column j at j*(m+1)), cs/sn[k][m], g[k][m+1],
// dots[k][2 (m+1)] with the pass-1 products at 0..j and the pass-2 products at m+1..m+1+j; nrm[k] the
// norm of w after both passes.
__global__ void k_gm_givens(int nrhs, int m, int j, const double* __restrict__ dots, const double* __restrict__ nrm,
                            double* __restrict__ Hs, double* __restrict__ cs, double* __restrict__ sn,
                            double* __restrict__ g, double* __restrict__ res)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nrhs) return;
    const double* d1 = dots + (int64_t)k * 2 * (m + 1);
    const double* d2 = d1 + (m + 1);
    double* H = Hs + (int64_t)k * (m + 1) * m + (int64_t)j * (m + 1);
    double* c = cs + (int64_t)k * m;
    double* s = sn + (int64_t)k * m;
    double* gk = g + (int64_t)k * (m + 1);
    for (int i = 0; i <= j; ++i) H[i] = d1[i] + d2[i];
    H[j + 1] = nrm[k];
    for (int i = 0; i < j; ++i) {
        const double a = H[i], b = H[i + 1];
        H[i] = c[i] * a + s[i] * b;
        H[i + 1] = -s[i] * a + c[i] * b;
    }
    const double a = H[j], b = H[j + 1];
    const double rr = hypot(a, b);
    const double cj = rr > 0.0 ? a / rr : 1.0, sj = rr > 0.0 ? b / rr : 0.0;
    c[j] = cj;
    s[j] = sj;
    H[j] = rr;
    H[j + 1] = 0.0;
    const double gj = gk[j];
    gk[j] = cj * gj;
    gk[j + 1] = -sj * gj;
    res[k] = fabs(gk[j + 1]);
}

// Start of a correction: g = (beta, 0, ...), beta = ||r|| (nrm[k]), res[k] = beta.
__global__ void k_gm_start(int nrhs, int m, const double* __restrict__ nrm, double* __restrict__ g,
                           double* __restrict__ res)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nrhs) return;
    double* gk = g + (int64_t)k * (m + 1);
    for (int i = 0; i <= m; ++i) gk[i] = 0.0;
    gk[0] = nrm[k];
    res[k] = nrm[k];
}

// y = R^{-1} g over the first nj columns (R the rotated, upper triangular Hessenberg matrix); a zero
// pivot (exhausted Krylov space of a converged column) gives y_i = 0.
__global__ void k_gm_backsolve(int nrhs, int m, int nj, const double* __restrict__ Hs, const double* __restrict__ g,
                               double* __restrict__ y)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nrhs) return;
    const double* H = Hs + (int64_t)k * (m + 1) * m;
    const double* gk = g + (int64_t)k * (m + 1);
    double* yk = y + (int64_t)k * m;
    for (int i = nj - 1; i >= 0; --i) {
        double acc = gk[i];
        for (int q = i + 1; q < nj; ++q) acc -= H[(int64_t)q * (m + 1) + i] * yk[q];
        const double piv = H[(int64_t)i * (m + 1) + i];
        yk[i] = piv != 0.0 ? acc / piv : 0.0;
    }
}

// One damped-Jacobi sweep of the preconditioner's smoother: Z += omega * R / diag(G), R = v - G z
// (the residual kernel's output), diag(G) read from the CSR row.
__global__ __launch_bounds__(kGThreads) void k_gm_jacobi(HierDev H, int nrhs, const double* __restrict__ R,
                                                         double omega, double* __restrict__ Z)
{
    const int k = blockIdx.y;
    const int r = blockIdx.x * kGThreads + threadIdx.x;
    if (r >= H.n) return;
    double d = 0.0;
    for (int e = H.rp[r]; e < H.rp[r + 1]; ++e)
        if (H.ci[e] == r) d = H.cv[e];
    const int64_t o = (int64_t)k * H.n + r;
    if (d > 0.0) Z[o] += omega * R[o] / d;
}

}  // namespace

static int gx(int n) { return (n + kGThreads - 1) / kGThreads; }

void launch_gm_jacobi(const HierDev& H, int nrhs, const double* R, double omega, double* Z, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_jacobi, dim3(gx(H.n), nrhs), dim3(kGThreads), 0, s, H, nrhs, R, omega, Z);
}

void launch_gm_dots(int n, int nrhs, int nv, const double* V, const double* W, double sgn, double* out, int ld_out,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_dots, dim3(nv, nrhs), dim3(kGThreads), 0, s, n, nrhs, V, W, sgn, out, ld_out, 0);
}

void launch_gm_norms(int n, int nrhs, const double* W, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_dots, dim3(1, nrhs), dim3(kGThreads), 0, s, n, nrhs, W, W, 1.0, out, 1, 1);
}

void launch_gm_update(int n, int nrhs, int nv, const double* V, const double* h, int ld_h, double sgn, double* W,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_update, dim3(gx(n), nrhs), dim3(kGThreads), 0, s, n, nrhs, nv, V, h, ld_h, sgn, W);
}

void launch_gm_scale(int n, int nrhs, const double* W, const double* nrm, int ld_nrm, double sgn, double* Vout,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_scale, dim3(gx(n), nrhs), dim3(kGThreads), 0, s, n, W, nrm, ld_nrm, sgn, Vout);
}

void launch_gm_givens(int nrhs, int m, int j, const double* dots, const double* nrm, double* Hs, double* cs,
                      double* sn, double* g, double* res, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_givens, dim3((nrhs + 63) / 64), dim3(64), 0, s, nrhs, m, j, dots, nrm, Hs, cs, sn, g, res);
}

void launch_gm_start(int nrhs, int m, const double* nrm, double* g, double* res, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_start, dim3((nrhs + 63) / 64), dim3(64), 0, s, nrhs, m, nrm, g, res);
}

void launch_gm_backsolve(int nrhs, int m, int nj, const double* Hs, const double* g, double* y, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_backsolve, dim3((nrhs + 63) / 64), dim3(64), 0, s, nrhs, m, nj, Hs, g, y);
}

}  // namespace hinv
