// Comparison baseline, not the paper's method: the sparse direct network solution that the
// inverse-based solver replaces (the LU-based solver of the paper's Introduction and Section V.B;
// G is SPD, so the factorization is Cholesky, G = P^T L L^T P).
//
//  host   : minimum-degree ordering on the graph of G, elimination tree, up-looking numeric
//           factorization (row k of L from a sparse triangular solve against the rows above it,
//           restricted to the row's elimination-tree reach), and the level schedules of the two
//           triangular solves (a row's level is one more than the deepest row it reads);
//  device : one workgroup per right-hand side sequence; x in LDS; per level the rows are split
//           over groups of 8 lanes (a strided dot product and three shuffle steps), one barrier
//           per level; forward solve with L by rows, backward with L^T by rows (L's columns).
#include <math.h>

#include <algorithm>
#include <memory>
#include <new>
#include <set>
#include <vector>

#include "hinv_internal.h"

using namespace hinv;

namespace {

constexpr int kCholThreads = 1024;
constexpr int kCholGroup = 8;                    // lanes per row
constexpr int kCholMaxN = 16384;                 // x in LDS

#define CHOL_TRY(expr)                                                                             \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return set_error(HINV_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct CholDev {
    int n;
    const int* perm;                             // [n] new row k holds old row perm[k]
    const int* f_lp;                             // forward levels: rows f_rows[f_lp[l] .. f_lp[l+1])
    const int* f_rows;
    const int* f_rp;                             // L by rows, strictly lower part: (col, val)
    const int* f_ci;
    const double* f_v;
    const int* b_lp;                             // backward levels
    const int* b_rows;
    const int* b_rp;                             // L^T by rows (L by columns), strictly upper part
    const int* b_ci;
    const double* b_v;
    const double* dinv;                          // 1 / L_kk
    int f_levels, b_levels;
};

struct CholHost {
    int n = 0;
    std::vector<int> perm;
    std::vector<int> f_lp, f_rows, f_rp, f_ci, b_lp, b_rows, b_rp, b_ci;
    std::vector<double> f_v, b_v, dinv;
    int64_t nnz_l = 0;
    double factor_flops = 0.0;
};

// Minimum degree on the elimination graph (ties to the lowest index), the textbook form.
std::vector<int> min_degree(const hinv_csr* G)
{
    const int n = G->n;
    std::vector<std::set<int>> adj(n);
    for (int r = 0; r < n; ++r)
        for (int e = G->row_ptr[r]; e < G->row_ptr[r + 1]; ++e)
            if (G->col_idx[e] != r && G->val[e] != 0.0) {
                adj[r].insert(G->col_idx[e]);
                adj[G->col_idx[e]].insert(r);
            }
    std::vector<char> done(n, 0);
    std::vector<int> order;
    order.reserve(n);
    for (int it = 0; it < n; ++it) {
        int v = -1;
        size_t best = 0;
        for (int i = 0; i < n; ++i)
            if (!done[i] && (v < 0 || adj[i].size() < best)) { v = i; best = adj[i].size(); }
        done[v] = 1;
        order.push_back(v);
        std::vector<int> nb(adj[v].begin(), adj[v].end());
        for (int a : nb) adj[a].erase(v);
        for (size_t i = 0; i < nb.size(); ++i)
            for (size_t j = i + 1; j < nb.size(); ++j) {
                adj[nb[i]].insert(nb[j]);
                adj[nb[j]].insert(nb[i]);
            }
        adj[v].clear();
    }
    return order;
}

hinv_status factorize(const hinv_csr* G, CholHost& C)
{
    const int n = G->n;
    C.n = n;
    C.perm = min_degree(G);
    std::vector<int> inv(n);
    for (int k = 0; k < n; ++k) inv[C.perm[k]] = k;
    // permuted lower triangle by rows: A(k, j), j <= k
    std::vector<std::vector<std::pair<int, double>>> arow(n);
    for (int r = 0; r < n; ++r)
        for (int e = G->row_ptr[r]; e < G->row_ptr[r + 1]; ++e) {
            const int k = inv[r], j = inv[G->col_idx[e]];
            if (j <= k) arow[k].push_back({j, G->val[e]});
        }
    // elimination tree (ancestor path compression)
    std::vector<int> par(n, -1), anc(n, -1);
    for (int k = 0; k < n; ++k)
        for (auto& [j0, v] : arow[k]) {
            (void)v;
            int j = j0;
            while (j != -1 && j < k) {
                const int nx = anc[j];
                anc[j] = k;
                if (nx == -1) { par[j] = k; break; }
                j = nx;
            }
        }
    // up-looking numeric factorization; L kept by columns (rows ascending) and by rows
    std::vector<std::vector<int>> lcol_r(n);
    std::vector<std::vector<double>> lcol_v(n);
    std::vector<std::vector<int>> lrow_c(n);
    std::vector<std::vector<double>> lrow_v(n);
    std::vector<double> diag(n), x(n, 0.0);
    std::vector<int> mark(n, -1);
    for (int k = 0; k < n; ++k) {
        double akk = 0.0;
        std::vector<int> pat;
        for (auto& [j, v] : arow[k]) {
            if (j == k) { akk += v; continue; }
            x[j] += v;
            for (int t = j; t != -1 && t < k && mark[t] != k; t = par[t]) {   // reach in the etree
                mark[t] = k;
                pat.push_back(t);
            }
        }
        std::sort(pat.begin(), pat.end());                                  // ascending = topological
        double d = akk;
        for (int j : pat) {
            const double lkj = x[j] / diag[j];
            x[j] = 0.0;
            const std::vector<int>& rows = lcol_r[j];
            const std::vector<double>& vals = lcol_v[j];
            for (size_t q = 0; q < rows.size(); ++q) x[rows[q]] -= vals[q] * lkj;   // rows i with j < i < k
            d -= lkj * lkj;
            lrow_c[k].push_back(j);
            lrow_v[k].push_back(lkj);
            C.factor_flops += 2.0 * (double)rows.size() + 3.0;
        }
        for (size_t q = 0; q < lrow_c[k].size(); ++q) {                     // column lists gain row k
            lcol_r[lrow_c[k][q]].push_back(k);
            lcol_v[lrow_c[k][q]].push_back(lrow_v[k][q]);
        }
        if (!(d > 0.0) || !isfinite(d))
            return set_error(HINV_E_NOT_SPD, "Cholesky pivot %d is %g: G is not positive definite", k, d);
        diag[k] = sqrt(d);
        C.factor_flops += 1.0;
    }
    // level schedules and device layouts
    std::vector<int> lf(n, 0), lb(n, 0);
    int nf = 0, nbk = 0;
    for (int k = 0; k < n; ++k) {
        int l = 0;
        for (int j : lrow_c[k]) l = std::max(l, lf[j] + 1);
        lf[k] = l;
        nf = std::max(nf, l + 1);
    }
    for (int k = n - 1; k >= 0; --k) {
        int l = 0;
        for (int i : lcol_r[k]) l = std::max(l, lb[i] + 1);
        lb[k] = l;
        nbk = std::max(nbk, l + 1);
    }
    auto schedule = [n](const std::vector<int>& lev, int nl, std::vector<int>& lp, std::vector<int>& rows) {
        lp.assign(nl + 1, 0);
        for (int k = 0; k < n; ++k) ++lp[lev[k] + 1];
        for (int l = 0; l < nl; ++l) lp[l + 1] += lp[l];
        rows.assign(n, 0);
        std::vector<int> fill(lp.begin(), lp.end() - 1);
        for (int k = 0; k < n; ++k) rows[fill[lev[k]]++] = k;
    };
    schedule(lf, nf, C.f_lp, C.f_rows);
    schedule(lb, nbk, C.b_lp, C.b_rows);
    C.f_rp.assign(n + 1, 0);
    C.b_rp.assign(n + 1, 0);
    for (int k = 0; k < n; ++k) {
        C.f_rp[k + 1] = C.f_rp[k] + (int)lrow_c[k].size();
        C.b_rp[k + 1] = C.b_rp[k] + (int)lcol_r[k].size();
        C.f_ci.insert(C.f_ci.end(), lrow_c[k].begin(), lrow_c[k].end());
        C.f_v.insert(C.f_v.end(), lrow_v[k].begin(), lrow_v[k].end());
        C.b_ci.insert(C.b_ci.end(), lcol_r[k].begin(), lcol_r[k].end());
        C.b_v.insert(C.b_v.end(), lcol_v[k].begin(), lcol_v[k].end());
    }
    C.dinv.resize(n);
    for (int k = 0; k < n; ++k) C.dinv[k] = 1.0 / diag[k];
    C.nnz_l = (int64_t)C.f_ci.size() + n;
    return HINV_OK;
}

struct Carve {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(size_t count)
    {
        off = (off + 255) / 256 * 256;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += sizeof(T) * (count > 0 ? count : 1);
        return p;
    }
};

void carve(const CholHost& C, Carve& A, CholDev& D)
{
    const int n = C.n;
    D.n = n;
    D.perm = A.take<int>(n);
    D.f_lp = A.take<int>(C.f_lp.size());
    D.f_rows = A.take<int>(n);
    D.f_rp = A.take<int>(n + 1);
    D.f_ci = A.take<int>(C.f_ci.size());
    D.f_v = A.take<double>(C.f_v.size());
    D.b_lp = A.take<int>(C.b_lp.size());
    D.b_rows = A.take<int>(n);
    D.b_rp = A.take<int>(n + 1);
    D.b_ci = A.take<int>(C.b_ci.size());
    D.b_v = A.take<double>(C.b_v.size());
    D.dinv = A.take<double>(n);
    D.f_levels = (int)C.f_lp.size() - 1;
    D.b_levels = (int)C.b_lp.size() - 1;
}

template <typename T>
hipError_t put(const T* dst, const std::vector<T>& src, hipStream_t s)
{
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync((void*)dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s);
}

// One level of a triangular solve: x[k] = (x[k] - sum_q v[q] x[ci[q]]) * dinv[k] for the level's rows.
__device__ __forceinline__ void chol_level(const int* rows, int r0, int r1, const int* rp, const int* ci,
                                           const double* v, const double* dinv, double* x)
{
    const int g = threadIdx.x / kCholGroup, lane = threadIdx.x % kCholGroup;
    constexpr int groups = kCholThreads / kCholGroup;
    for (int q0 = r0; q0 < r1; q0 += groups) {
        const int q = q0 + g;
        double acc = 0.0;
        int k = -1;
        if (q < r1) {
            k = rows[q];
            for (int e = rp[k] + lane; e < rp[k + 1]; e += kCholGroup) acc += v[e] * x[ci[e]];
        }
        acc += __shfl_xor(acc, 4, kCholGroup);
        acc += __shfl_xor(acc, 2, kCholGroup);
        acc += __shfl_xor(acc, 1, kCholGroup);
        if (q < r1 && lane == 0) x[k] = (x[k] - acc) * dinv[k];
    }
}

__global__ __launch_bounds__(kCholThreads) void k_chol_solve(CholDev D, const double* B, double* X, int nrhs, int ld)
{
    extern __shared__ double xs[];
    const int n = D.n;
    for (int r = 0; r < nrhs; ++r) {
        const double* b = B + (int64_t)r * ld;
        for (int k = threadIdx.x; k < n; k += kCholThreads) xs[k] = b[D.perm[k]];
        __syncthreads();
        for (int l = 0; l < D.f_levels; ++l) {
            chol_level(D.f_rows, D.f_lp[l], D.f_lp[l + 1], D.f_rp, D.f_ci, D.f_v, D.dinv, xs);
            __syncthreads();
        }
        for (int l = 0; l < D.b_levels; ++l) {
            chol_level(D.b_rows, D.b_lp[l], D.b_lp[l + 1], D.b_rp, D.b_ci, D.b_v, D.dinv, xs);
            __syncthreads();
        }
        double* xo = X + (int64_t)r * ld;
        for (int k = threadIdx.x; k < n; k += kCholThreads) xo[D.perm[k]] = xs[k];
        __syncthreads();
    }
}

}  // namespace

struct chol_ctx {
    CholHost C;
    CholDev D{};
};

extern "C" {

hinv_status chol_workspace_size(const hinv_csr* G, size_t* bytes)
{
    if (!bytes) return set_error(HINV_E_INVALID, "bytes is NULL");
    hinv_status st0 = validate_csr(G);
    if (st0 != HINV_OK) return st0;
    if (G->n > kCholMaxN) return set_error(HINV_E_INVALID, "n %d above %d", G->n, kCholMaxN);
    std::unique_ptr<chol_ctx> c(new (std::nothrow) chol_ctx);
    if (!c) return set_error(HINV_E_NO_MEMORY, "host allocation failed");
    hinv_status st = factorize(G, c->C);
    if (st != HINV_OK) return st;
    Carve A;
    carve(c->C, A, c->D);
    *bytes = A.off + 256;
    return HINV_OK;
}

hinv_status chol_create(const hinv_csr* G, void* d_ws, size_t ws_bytes, void* stream, chol_handle* out)
{
    if (!out) return set_error(HINV_E_INVALID, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    hinv_status st = chol_workspace_size(G, &need);
    if (st != HINV_OK) return st;
    if (!d_ws || ws_bytes < need) return set_error(HINV_E_NO_MEMORY, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    std::unique_ptr<chol_ctx> c(new (std::nothrow) chol_ctx);
    if (!c) return set_error(HINV_E_NO_MEMORY, "host allocation failed");
    st = factorize(G, c->C);
    if (st != HINV_OK) return st;
    Carve A;
    A.base = (char*)d_ws;
    carve(c->C, A, c->D);
    hipStream_t s = (hipStream_t)stream;
    const CholHost& C = c->C;
    CholDev& D = c->D;
    CHOL_TRY(put(D.perm, C.perm, s));
    CHOL_TRY(put(D.f_lp, C.f_lp, s)); CHOL_TRY(put(D.f_rows, C.f_rows, s)); CHOL_TRY(put(D.f_rp, C.f_rp, s));
    CHOL_TRY(put(D.f_ci, C.f_ci, s)); CHOL_TRY(put(D.f_v, C.f_v, s));
    CHOL_TRY(put(D.b_lp, C.b_lp, s)); CHOL_TRY(put(D.b_rows, C.b_rows, s)); CHOL_TRY(put(D.b_rp, C.b_rp, s));
    CHOL_TRY(put(D.b_ci, C.b_ci, s)); CHOL_TRY(put(D.b_v, C.b_v, s));
    CHOL_TRY(put(D.dinv, C.dinv, s));
    CHOL_TRY(hipStreamSynchronize(s));
    *out = c.release();
    return HINV_OK;
}

hinv_status chol_solve(chol_handle h, const double* d_b, double* d_x, int32_t nrhs, int32_t ld, void* stream)
{
    if (!h) return set_error(HINV_E_INVALID, "handle is NULL");
    const CholDev& D = h->D;
    if (nrhs < 0 || ld < D.n) return set_error(HINV_E_INVALID, "nrhs %d / ld %d invalid for n %d", nrhs, ld, D.n);
    if (nrhs == 0) return HINV_OK;
    if (!d_b || !d_x) return set_error(HINV_E_INVALID, "NULL vector");
    const size_t lds = sizeof(double) * (size_t)D.n;
    CHOL_TRY(hipFuncSetAttribute((const void*)k_chol_solve, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_chol_solve, dim3(1), dim3(kCholThreads), lds, (hipStream_t)stream, D, d_b, d_x, nrhs, ld);
    CHOL_TRY(hipGetLastError());
    return HINV_OK;
}

hinv_status chol_get_info(chol_handle h, chol_info_t* out)
{
    if (!h || !out) return set_error(HINV_E_INVALID, "NULL argument");
    const CholHost& C = h->C;
    out->n = C.n;
    out->nnz_l = C.nnz_l;
    out->fwd_levels = (int64_t)C.f_lp.size() - 1;
    out->bwd_levels = (int64_t)C.b_lp.size() - 1;
    out->solve_flops = 4.0 * (double)(C.nnz_l - C.n) + 2.0 * C.n;
    out->factor_flops = C.factor_flops;
    return HINV_OK;
}

hinv_status chol_destroy(chol_handle h)
{
    delete h;
    return HINV_OK;
}

}  // extern "C"
