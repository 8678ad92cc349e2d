// Internal structures of libhinv (host orchestration <-> HIP kernels).
//
// Bus order.  The library renumbers buses so that every tree node owns a
// contiguous row range [lo, lo+n): leaves in depth-first order, buses of a
// leaf in increasing original index.  perm[new] = old, iperm[old] = new.
//
// Stored exact inverse (FP64 master, optional low-precision copy):
//   leaf blocks   B_l^{-1}, n_l x n_l, column-major (ld = n_l)
//   internal node t with children c_1..c_k and cut lines (a_j, b_j, g_j):
//     U_t has 2 columns per cut line, sqrt|G_ab| e_a and sqrt|G_ab| e_b;
//     coupling  G_t - blockdiag(G_c) = U_t C_t U_t^T, C_t pairs the two
//     columns of a line with sign(G_ab);
//     Z_t = blockdiag(G_c^{-1}) U_t, stored per child as a "panel": the rows
//     of child c times the columns whose endpoint lies in c, column-major;
//     S_t = C_t + U_t^T Z_t (m_t x m_t), stored as S_t^{-1}, column-major.
//   Then G_t^{-1} x = v0 - Z_t S_t^{-1} U_t^T v0 with v0 = blockdiag(G_c^{-1}) x.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hinv.h"

namespace hinv {

constexpr int kMaxLeaf = HINV_MAX_LEAF;
constexpr int kMaxModRank = 16;
constexpr int kBlock = 256;

// Device view of the hierarchy (kernel argument, all pointers into the workspace).
struct HierDev {
    int n, n_leaves, n_internal, n_levels, n_cols, anc_stride, max_cols, max_pan_rows;
    // leaves
    const int* leaf_lo;
    const int* leaf_n;
    const int64_t* leaf_off;   // element offset of the block
    const int* leaf_anc;       // [n_leaves * anc_stride] internal ancestors, nearest first, -1 padded
    const int* row_leaf;       // [n] leaf of each (new-order) row
    // internal nodes, ordered by level (height) then index
    const int* node_lo;
    const int* node_n;
    const int* node_m;
    const int* node_col0;
    const int64_t* node_soff;  // offset of S^{-1}
    const int* node_pan0;
    const int* node_npan;
    const int* node_level;
    // child panels
    const int* pan_lo;
    const int* pan_n;
    const int* pan_col0;
    const int* pan_m;
    const int64_t* pan_zoff;
    // coupling columns (global numbering, grouped by node then panel)
    const int* col_row;
    const double* col_w;
    const int* col_partner;
    const double* col_sign;
    const int* col_pan;
    // per level (1..n_levels): [lvl_x[l-1], lvl_x[l]) ranges
    const int* lvl_node;
    const int* lvl_pan;
    const int* lvl_col;
    // G in the new order (CSR)
    const int* rp;
    const int* ci;
    const double* cv;
    // values
    double* blk;
    double* Z;
    double* Sinv;
    float* blk32;
    float* Z32;
    float* Sinv32;
};

// Line changes (Sherman-Morrison-Woodbury) for n_sets independent sets
// (a standalone hierarchy has one set; an EMT batch one per case).
struct ModDev {
    int n_sets, R, n;
    const int* count;       // [n_sets] changes stored
    const int* a;           // [n_sets*R] new-order row, -1 unused
    const int* b;           // [n_sets*R] new-order row or -1 (ground)
    const double* dg;       // [n_sets*R]
    const int* act;         // [n_sets*R] first step the change is active (sorted per set)
    double* U;              // [n_sets*R*n] u_j = G0^{-1} w_j
    float* U32;             // low-precision copy
    double* Cinv;           // [n_sets*R*R*R]: inverse of the leading r x r capacitance, r = 1..R
};

// EMT network and per-case state (new bus order), kernel argument.
struct EmtDev {
    int n, nbr, n_cases, R;
    double dt, omega;
    const int* fr;          // [nbr] new-order endpoints
    const int* to;
    const double* g;        // branch companion conductance 1/(R + 2L/dt)
    const double* alpha;    // history weight g (2L/dt - R)
    const double* gC;       // [n] shunt companion conductance 2C/dt
    const int* inc_ptr;     // [n+1] incident branches of each bus
    const int* inc_br;
    const int* src_ptr;     // [n+1] sources of each bus
    const double* src_amp;
    const double* src_ph;
    const int* loss_cnt;    // [n_cases]
    const int* loss_step;   // [n_cases*R] sorted by step
    const int* loss_br;     // [n_cases*R]
    const int* perm;        // new -> caller bus index
    double* h;              // [2][n_cases*nbr] branch history, ping-pong by step parity
    double* hC;             // [n_cases*n]
    double* b;              // [n_cases*n] right-hand side of the current step
    double* v;              // [n_cases*n]
    int64_t* step;          // next step to compute
    unsigned int* done;     // block counter for the step advance
};

// Where emt_step records v and b (device struct, updated per call).
struct RecParams {
    double* v;
    double* b;
    int64_t step0;
    int64_t nsteps;
};

// Host-side per-level launch sizes (level l = 1..n_levels at index l-1).
struct LevelHost {
    int nnodes, npan, ncols, max_m, max_pan_rows;
};

// Status flag bits written by kernels.
enum : int { kFlagNotSPD = 1, kFlagSingular = 2, kFlagNaN = 4, kFlagNoConv = 8 };

// ---------------- kernel launchers (k_build.hip / k_apply.hip / k_emt.hip)
void launch_leaf_inverse(const HierDev& H, int* flags, hipStream_t s);
void launch_build_z(const HierDev& H, int level, int ncols, hipStream_t s);
void launch_fill_s(const HierDev& H, int level, int nnodes, hipStream_t s);
void launch_gj_level(const HierDev& H, int level, int nnodes, int m_max, double* colbuf, int* ipiv, int* flags,
                     hipStream_t s);
void launch_to_f32(const double* src, float* dst, int64_t count, hipStream_t s);

void launch_permute_in(int n, int nrhs, const int* perm, const double* src, int ld, double* X, hipStream_t s);
void launch_permute_out(int n, int nrhs, const int* perm, const double* X, double* dst, int ld, hipStream_t s);
// Hierarchy apply: X (n x nrhs, ld n, new order) -> Xout = G0^{-1} X.  Y: scratch [nrhs * n_cols].
void launch_apply(const HierDev& H, const LevelHost* lv, int prec, const double* X, double* Xout, double* Y,
                  int nrhs, hipStream_t s);
// v += d (column k of nrhs).  With stats: folds max|d|/max|v| of column k into
// stats[k] (non-negative doubles compared as integers) and raises kFlagNoConv
// in *flags when it exceeds rel_tol (kFlagNaN when not finite).
void launch_axpy_stats(int n, int nrhs, double* V, const double* D, unsigned long long* stats, double rel_tol,
                       int* flags, hipStream_t s);
// SMW correction of v0 (in place) with the changes active at *step_ptr
// (step_ptr NULL: all stored changes).  Column k of V uses set set0 + k*set_stride.
void launch_smw_apply(const ModDev& M, int prec, double* V, int nrhs, int set0, int set_stride,
                      const int64_t* step_ptr, hipStream_t s);
// Capacitance inverses of every prefix of set k's stored changes (FP64).
void launch_smw_capacitance(const ModDev& M, int* flags, hipStream_t s);
// r = b - G_step v with the changes active at *step_ptr (NULL: all); column k uses set k*set_stride.
void launch_residual(const HierDev& H, const ModDev& M, const double* Bv, const double* V, double* Rv,
                     int nrhs, int set_stride, const int64_t* step_ptr, hipStream_t s);

void launch_emt_init(const EmtDev& E, hipStream_t s);
// Stream-ordered update of the record parameters (kernel argument, no host buffer to keep alive).
void launch_set_rec(RecParams* d, const RecParams& val, hipStream_t s);
// History update with v_n and assembly of b_{n+1}; records; advances *E.step.
void launch_emt_history(const EmtDev& E, const RecParams* rec, hipStream_t s);

}  // namespace hinv
