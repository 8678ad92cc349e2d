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
#include <vector>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hinv.h"

namespace hinv {

constexpr int kMaxLeaf = HINV_MAX_LEAF;
constexpr int kTeamMaxLevels = 4;     // coupling levels of a tree the team engine takes
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
    // fused-kernel lookups
    const int* row_lo;         // [n] first row of the row's leaf
    const int* row_nl;         // [n] size of the row's leaf
    const int64_t* row_boff;   // [n] offset of the row's entry in column 0 of its leaf block
    const int* col_node;       // [n_cols] internal node of each column
    const int* lvl_frow;       // [n_levels+1] flat panel-row ranges per level
    const int* frow_pan;       // [total panel rows] panel of each flat panel row
    const int* pan_frow0;      // [n_pan] first flat row of each panel
    const int* col_m;          // [n_cols] size m of the column's node
    const int* col_c0;         // [n_cols] first column of the column's node
    const int64_t* col_soff;   // [n_cols] S^{-1} offset of the column's node + (column - first column)
    const int64_t* frow_z;     // [flat rows] offset of the row's entry in column 0 of its Z panel
    const int* frow_pn;        // [flat rows] panel rows (column stride)
    const int* frow_pm;        // [flat rows] panel columns
    const int* frow_pc;        // [flat rows] panel's first global column
    const int* frow_row;       // [flat rows] new-order row
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
    uint16_t* blk16;           // BF16 copies (round to nearest even)
    uint16_t* Z16;
    uint16_t* Sinv16;
    uint8_t* blk8;             // OCP FP8 E4M3 copies, one E8M0 scale per 32 consecutive entries
    uint8_t* Z8;
    uint8_t* Sinv8;
    uint8_t* blk8s;
    uint8_t* Z8s;
    uint8_t* Sinv8s;
};

// Element accessors for the stored-inverse formats (value as the accumulator type).
struct StF64 {
    const double* p;
    __device__ __forceinline__ double operator[](int64_t i) const { return p[i]; }
};
struct StF32 {
    const float* p;
    __device__ __forceinline__ float operator[](int64_t i) const { return p[i]; }
};
struct StBF16 {
    const uint16_t* p;
    __device__ __forceinline__ float operator[](int64_t i) const { return __uint_as_float((uint32_t)p[i] << 16); }
};
// OCP E4M3: sign, 4-bit exponent (bias 7), 3-bit mantissa; exponent 0 is subnormal.
__device__ __forceinline__ float e4m3_to_float(uint8_t b)
{
    const int e = (b >> 3) & 15, m = b & 7;
    const float mag = e == 0 ? ldexpf((float)m, -9) : ldexpf(1.0f + 0.125f * (float)m, e - 7);
    return (b & 0x80) ? -mag : mag;
}
struct StFP8 {
    const uint8_t* p;
    const uint8_t* e;          // E8M0 scale exponents (2^(e-127)) of each 32-entry group
    __device__ __forceinline__ float operator[](int64_t i) const
    {
        return ldexpf(e4m3_to_float(p[i]), (int)e[i >> 5] - 127);
    }
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
    // Three-phase line changes: changes 3g, 3g+1, 3g+2 of a set are the phases of one line, whose 3x3
    // coupling D (G <- G + W D W^T, W the three phase-difference vectors) is not diagonal.  Row p of D
    // and of D^{-1} for change 3g+p (null / 0 for single-phase sets, where D = diag(dg)).
    int grp3;
    const double* d3;       // [n_sets*R*3]
    const double* dinv3;    // [n_sets*R*3]
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
    // three-phase networks: rows are bus phases, branch 3l+p is phase p of line l, whose companion is
    // the 3x3 admittance Y3[l] with history weight A3[l] (row-major, phase order); null otherwise
    const double* Y3;       // [nbr/3 * 9]
    const double* A3;       // [nbr/3 * 9]
};

// Where emt_step records v and b (device struct, updated per call).
struct RecParams {
    double* v;
    double* b;
    int64_t step0;
    int64_t nsteps;
};

// Fused stepping launch parameters.
struct RunParams {
    int64_t step0;
    int n_steps;
    int max_refine;
    double rel_tol;
    int warm;
    double* v_rec;
    double* b_rec;
    int* flags;
    unsigned long long* stats;     // [n_cases] largest final correction ratio
    unsigned long long* applies;   // [n_cases] applies performed
    int64_t* clk;                  // optional: wall clock after each step of case 0
    int64_t clk_cap;
    int64_t rec_step0;             // v_rec/b_rec row j holds step rec_step0 + j, j < rec_cap
    int64_t rec_cap;
};

// One slot of a serving launch: one case of an EMT handle (k_run.hip).
struct ServeSlot {
    EmtDev E;
    HierDev H;
    ModDev M;
    int k;
    int gvec;                      // case vectors in global scratch instead of LDS
    double* gscr;                  // [4*n] scratch of the case (gvec)
    double* v_rec;
    int64_t rec_step0;
    int64_t rec_cap;
    int max_refine;
    double rel_tol;
    int* flags;
    unsigned long long* stats;
    unsigned long long* applies;
};

// Team stepping (k_team.hip): one workgroup per leaf of a single case.  All
// per-workgroup tables use fixed strides (the maxima over workgroups) so the
// LDS layout is the same in every workgroup.  "Combined" indices: own rows of
// the leaf are 0..nl-1, the workgroup's external rows ("X rows": coupling
// column endpoints, tie-line neighbours, line-loss endpoints) are nl + x.
struct TeamDev {
    int T, H, NL, NX, NB, NE, NI, NS, XZ, ZO;
    int nc, sent, NY;    // coupling columns, S^{-1} entries in LDS, most columns whose y a workgroup computes
    const int* csop;     // [T*nc] LDS offset of the column's row of its node's S^{-1} (entry p at csop + p*cld), -1: y not needed
    const int* cld;      // [T*nc] leading dimension of that node's block of needed rows in the workgroup's LDS
    const int* ylist;    // [T*nc] columns whose y the workgroup computes (first w_ny entries)
    const int* w_ny;     // [T]
    const int* w_lo;
    const int* w_nl;
    const int* w_nx;
    const int* w_nb;
    const int* xrow;     // [T*NX] new-order row of each X row (sorted)
    const int* w_nxu;    // [T] X rows whose final values the workgroup uses
    const int* xupd;     // [T*NX] their X positions: G neighbours of own rows and line-loss endpoints
    const int* uzo;      // [T*NX*H] offset of those rows' Z values at each level in LDS, -1: none
    int XZU;             // LDS entries of those Z values
    const int* xzo;      // [T*NX*H] offset of the row's Z values at level h in the xz region, -1: none
    const int* xpm;      // [T*NX*H] columns of that panel
    const int* xpc;      // [T*NX*H] first global column of that panel
    const int* ozo;      // [T*H] offset of the own rows' Z values at level h in the zown region, -1: none
    const int* opm;
    const int* opc;
    const int* opan;     // [T*H] panel index of the own rows at level h, -1: none
    const int* xpan;     // [T*NX*H] panel index of each X row at level h, -1: none
    const int* xpos;     // [T*n_cols] X position of each coupling column's row
    const int* orp;      // [T*(NL+1)] own CSR rows of G, combined column indices
    const int* ocol;     // [T*NE]
    const double* oval;
    const int* bglob;    // [T*NB] incident branches: global id, endpoints (combined), owner flag
    const int* bf;
    const int* bt;
    const int* bown;
    const double* bg;
    const double* bal;
    const int* iptr;     // [T*(NL+1)] incident local branches of each own row
    const int* ibr;      // [T*NI]
    const int* sptr;     // [T*(NL+1)] sources of each own row
    const double* samp;  // [T*NS]
    const double* sph;
    unsigned int* sync;  // [T] barrier epoch flag of each workgroup
    double* X0;          // [2*n] exchange of leaf results (double-buffered by apply parity)
    double* VM;          // [2*T] each workgroup's max |v| (same buffering)
    // Coupling levels in two phases.  With u_g the leaf-apply value at column g's row,
    // s_g = w_g u_g - sum_k a_g[k] u_{alo_g + k}, where the row a_g folds the corrections that the
    // lower levels' y would make to that row (the Z panels of the row at the lower levels through
    // their S^{-1}), then y = S^{-1} s for every level at once.  a_g is the same for every
    // workgroup; launch_team_acoef computes it on the device from the FP64 hierarchy.
    int nA;              // entries of all rows a_g
    const int* aoff;     // [n_cols] offset of a_g
    const int* alo;      // [n_cols] first column of a_g
    const int* alen;     // [n_cols] length of a_g (0 on the lowest level)
    const int* cpan;     // [n_cols*H] panel of the column's row at each lower level, -1: none
    double* acoef;       // [nA] FP64 rows a_g
    float* acoef32;      // [nA] FP32 copy
    double* am;          // [n_cols*n_cols] scratch: off-diagonal part of s as a map from u
    double* bm;          // [n_cols*n_cols] scratch: y as a map from u
};

// Panel stepping (k_panel.hip): cases that share one base network advance in
// panels of kPanelCases; a team of one workgroup per leaf owns one panel and
// applies the leaf blocks to the panel as one matrix product.  Per-leaf tables
// use fixed strides.  X rows of a leaf: its buses' neighbours through G in
// other leaves (the same in every team); each is the row of a coupling column.
// Combined index: own row r -> r, X row x -> nl + x.  Vectors are row-major
// [row][case].
//
// Coupling levels in one map: the y of every coupling column is a linear map
// of u, the leaf-apply values at the column rows (y = M u, M built on the
// device from the FP64 Z panels, S^{-1} and column weights).  A workgroup
// computes the y of the columns its own rows and X rows apply ("slots",
// grouped by the columns' dependency range and padded to 16-row tiles) as
// MFMA tasks; a range's k-steps are split into tasks of at most
// kPanelYChain k-steps by a rule that depends on the range alone, so every
// workgroup computing a column's y runs the same operations, and an X row's
// value is formed exactly as its owner forms it.
constexpr int kPanelCases = 16;
constexpr int kPanelMaxRank = 2;
constexpr int kPanelMaxLeaf = 96;    // rows of a leaf
constexpr int kPanelMaxCols = 256;   // coupling columns of the tree
constexpr int kPanelMaxX = 128;      // X rows of a leaf
constexpr int kPanelYChain = 14;     // most k-steps (of 4 columns) of one y task
constexpr int kPanelYTasksPerWave = 2;
constexpr int kPanelWaves = 8;       // wavefronts of a panel workgroup
struct PanelDev {
    int T, H, NL, NLp, NX, NB, NE, NI, NS, XZ, ZO, nc, ncp, n_teams, team0;
    int NY;              // y slots of a workgroup (multiple of 16), most over the leaves
    int NT;              // y tasks of a workgroup, most over the leaves
    int MF;              // M fragment entries of a workgroup (multiple of 64), most over the leaves
    int NP;              // published (row, column) pairs of a leaf, most over the leaves
    int ysep;            // 1: the y tasks' results have an LDS region of their own (else they overwrite u)
    size_t imgb;         // bytes of one leaf's image of its LDS tables
    unsigned char* img;  // [T*imgb] the leaves' images (k_panel_image), copied into LDS at every launch
    int teams_per_launch;    // teams co-resident in one cooperative launch
    unsigned int epoch0;     // barrier epochs of earlier launches (flags are never reset between launches)
    // per leaf l
    const int* w_lo;
    const int* w_nl;
    const int* w_nb;
    const int* w_nx;
    const int* w_ny;     // [T] slots in use (padded)
    const int* w_nt;     // [T] y tasks
    const int* ozo;      // [T*H] offset of the own rows' Z values at level h in the zown region, -1: none
    const int* opm;
    const int* ops;      // [T*H] slot of the level-h panel's first column
    const int* opan;
    const int* orp;      // [T*(NL+1)] own CSR rows of G, combined column indices
    const int* ocol;     // [T*NE]
    const double* oval;
    const int* bglob;    // [T*NB] incident branches: global id, endpoints (combined), owner flag
    const int* bf;
    const int* bt;
    const int* bown;
    const double* bg;
    const double* bal;
    const int* iptr;     // [T*(NL+1)] incident local branches of each own row
    const int* ibr;      // [T*NI] local branch index, or its complement where the row is the branch's to-bus
    const int* hbft;     // [T*NB] the branch's endpoints (combined indices), from | to << 16
    const int* hlost;    // [n_teams*T*NB*kPanelCases] first step from which the branch is lost for the case
    const int* sptr;     // [T*(NL+1)] sources of each own row
    const double* samp;  // [T*NS]
    const double* sph;
    const int* w_np;     // [T] published (own row, column) pairs
    const int* pubr;     // [T*NP] own row of each pair
    const int* pubg;     // [T*NP] coupling column of each pair
    const int* xrow;     // [T*NX] new-order row of each X row
    const int* xcol;     // [T*NX] a coupling column whose row is the X row (its exchange index)
    const int* w_xz;     // [T] Z values of the X rows
    const int* xzsrc;    // [T*XZ] index of each of them in the hierarchy's Z array
    const int* xzo;      // [T*NX*H] offset of the X row's Z values at level h in the xz region, -1: none
    const int* xpm;
    const int* xps;      // [T*NX*H] slot of the panel's first column
    const int* xpan;
    const int* yslot;    // [T*NY] coupling column of each slot, -1: padding
    const int* tk0;      // [T*NT] y task: first absolute k-step, k-steps, fragment offset, tile
    const int* tnk;
    const int* tfo;
    const int* ttile;
    const int* ttp;      // [T*(NY/16+1)] tasks of tile t: ttl[ttp[t] .. ttp[t+1]) in k order
    const int* ttl;      // [T*NT]
    const int* wtask;    // [T*kPanelWaves*kPanelYTasksPerWave] tasks of each wavefront, -1: none
    const double* mfr;   // [T*MF] M as A fragments of the y tasks (FP64)
    const float* mfr32;  // [T*MF] FP32 copy
    // per (team, leaf) pair tw = team*T + l
    const int* lpa;      // [n_teams*T*kPanelCases*R] combined index of each change's endpoints (-1: not a row here)
    const int* lpb;
    // coupling map (device build of M)
    const int* cpan;     // [nc*H] panel of the column's row at each lower level, -1: none
    double* am;          // [nc*nc] scratch of the map build
    double* bm;          // [nc*nc] M (y = M u)
    unsigned int* sync;  // [n_teams*T] barrier epoch flags
    double* X0;          // [n_teams][2][nc][kPanelCases] exchange of leaf products at the column rows
    double* SP;          // [n_teams][2][T][R][kPanelCases] each workgroup's share of w^T v0 = u^T x per change
    double* VM;          // [n_teams][2][T][kPanelCases] each workgroup's max |v| per case
};

// Level stepping (k_level.hip): one case, one workgroup per leaf, for trees whose coupling
// levels do not fit every workgroup's LDS.  Every row has one owner; each coupling column is
// owned by the workgroup that owns its endpoint row, and owns the matching row of its node's
// S^{-1}.  Per apply: leaf product of the own rows; per level, the owners publish s, a barrier,
// the owners publish y = S^{-1} s, a barrier, and every workgroup corrects its own rows; then
// the own rows' values are published and a last barrier lets every workgroup read its X rows
// (neighbours through G, line-loss endpoints).  Per-leaf tables use fixed strides; combined
// index: own row r -> r, X row x -> nl + x.
struct LevelDev {
    int T, H, NL, NX, NB, NE, NI, NS, ZO, NO, SO, PM;
    const int* w_lo;
    const int* w_nl;
    const int* w_nb;
    const int* w_nx;
    const int* ozo;      // [T*H] offset of the own rows' Z values at level h in the zown region, -1: none
    const int* opm;
    const int* opc;
    const int* opan;
    const int* optr;     // [T*(H+1)] owned columns of level h: entries optr[h-1] .. optr[h]
    const int* ocl;      // [T*NO] owned column (global index)
    const int* orow;     // [T*NO] own row of the column's endpoint
    const int* osoff;    // [T*NO] LDS offset of the column's S^{-1} row
    const int* xrow;     // [T*NX] new-order row of each X row
    const int* orp;      // [T*(NL+1)] own CSR rows of G, combined column indices
    const int* ocol;     // [T*NE]
    const double* oval;
    const int* bglob;    // [T*NB] incident branches: global id, endpoints (combined), owner flag
    const int* bf;
    const int* bt;
    const int* bown;
    const double* bg;
    const double* bal;
    const int* iptr;     // [T*(NL+1)] incident local branches of each own row
    const int* ibr;      // [T*NI]
    const int* sptr;     // [T*(NL+1)] sources of each own row
    const double* samp;  // [T*NS]
    const double* sph;
    const int* lpa;      // [T*R] combined index of each change's endpoints (-1: ground / unused)
    const int* lpb;
    unsigned int* sync;  // [T] barrier epoch flags
    double* Sx;          // [2*n_cols] exchange of s at the top level (double-buffered by apply parity)
    unsigned long long* SL;   // [2*n_cols] s of the lower levels as tagged words (tag as for YL)
    unsigned long long* YL;   // [2*n_cols] y of every column as two tagged words (tagged_store / tagged_load),
                              // tag (apply index of the case's run) * 8 + level; read without a barrier
    double* V1;          // [n] exchange of the own rows' values at the end of an apply
    unsigned long long* VL;   // [2*n] the same as tagged words (tag: the apply's y tag, level 0), for applies
                              // that end without a barrier
    double* VM;          // [T] max |v| of each workgroup (convergence norm)
};

// One case of a launch of several level-stepped cases (serving).
struct LevelCase {
    LevelDev D;
    EmtDev E;
    HierDev H;
    ModDev M;
    RunParams P;
    int wg0;             // first workgroup of the case within its launch
    int pad;
};

// Host-side per-level launch sizes (level l = 1..n_levels at index l-1).
struct LevelHost {
    int nnodes, npan, ncols, max_m, max_pan_rows;
};

// Status flag bits written by kernels.
enum : int { kFlagNotSPD = 1, kFlagSingular = 2, kFlagNaN = 4, kFlagNoConv = 8, kFlagBarrier = 16, kFlagTeamRow = 32 };

// The library's error string (hinv_last_error); returns st.
hinv_status set_error(hinv_status st, const char* fmt, ...);
// Symmetric CSR with sorted columns, finite values and a positive diagonal (else INVALID / NOT_SPD).
hinv_status validate_csr(const hinv_csr* G);

// ---------------- kernel launchers (k_build.hip / k_apply.hip / k_emt.hip)
// Builders of the stored inverse.  list (device): the leaves / columns / nodes to (re)build, count
// entries; NULL: every leaf, or every column / node of the level (ncols / nnodes of them).
void launch_leaf_inverse(const HierDev& H, int* flags, hipStream_t s, const int* list = nullptr, int count = 0);
void launch_build_z(const HierDev& H, int level, int ncols, hipStream_t s, const int* list = nullptr);
void launch_fill_s(const HierDev& H, int level, int nnodes, int m_max, hipStream_t s, const int* list = nullptr,
                   bool coupling_only = false);
// S^{-1} of the listed nodes (order <= kNodeGjMax each): assembly and inversion in one workgroup.
constexpr int kNodeGjMax = 128;
void launch_node_inverse(const HierDev& H, const int* list, int count, int* flags, hipStream_t s);
// S^{-1} of the listed nodes of order kNodeGjMax < m <= kGjTeamMax (m_of: their orders, host):
// blocked Gauss-Jordan by a team of workgroups per node, cooperative launches.  xb / sync:
// device exchange doubles and barrier words, at least what gj_team_sizes reports for m_of.
constexpr int kGjTeamMax = 1024;
hipError_t launch_gj_team(const HierDev& H, const int* list, const std::vector<int>& m_of, double* xb,
                          unsigned int* sync, int* flags, hipStream_t s);
void gj_team_sizes(const std::vector<int>& m_of, int64_t* xb_doubles, int64_t* sync_words);
void launch_gj_level(const HierDev& H, int level, int nnodes, int m_max, double* colbuf, int* ipiv, int* flags,
                     hipStream_t s, const int* list = nullptr);
void launch_to_f32(const double* src, float* dst, int64_t count, hipStream_t s);
void launch_to_bf16(const double* src, uint16_t* dst, int64_t count, hipStream_t s);
// E4M3 with one E8M0 scale per 32 entries (count rounded up to whole groups in `scale`)
void launch_to_fp8(const double* src, uint8_t* dst, uint8_t* scale, int64_t count, hipStream_t s);

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
// Re-assemble the current step's b of case k (after a loss was added for this step).
void launch_emt_rebuild_rhs(const EmtDev& E, int k, hipStream_t s);
// Stream-ordered update of the record parameters (kernel argument, no host buffer to keep alive).
void launch_set_rec(RecParams* d, const RecParams& val, hipStream_t s);
// Team stepping (k_team.hip): LDS bytes of the layout, and the launch.
size_t team_lds_bytes(const TeamDev& T, const HierDev& H, int R, int prec, int warm);
hipError_t launch_team_acoef(const TeamDev& T, const HierDev& H, hipStream_t s);
// y of every coupling column as a map of u (y = bm u; am: scratch), bottom-up over the levels from the
// FP64 Z panels, S^{-1} and column weights (cpan: [nc*Hn] panel of the column's row at each lower level).
hipError_t launch_coupling_map(const HierDev& H, int Hn, int nc, const int* cpan, double* am, double* bm,
                               hipStream_t s);
hipError_t launch_emt_team(const TeamDev& T, const EmtDev& E, const HierDev& H, const ModDev& M, const RunParams& P,
                           int prec, hipStream_t s);
// Panel stepping (k_panel.hip): LDS bytes of the layout, and the launch (all
// teams, in as many consecutive cooperative launches as residency requires).
size_t panel_lds_bytes(const PanelDev& D, int R, int prec, int warm);
// Launch set-up of the panel kernel for this layout (dynamic LDS limit, teams per cooperative launch).
hipError_t panel_setup(PanelDev& D, int R, int prec, int warm);
// M as the y tasks' A fragments (D.mfr, D.mfr32) from D.bm; after launch_coupling_map.
hipError_t launch_panel_mfrag(const PanelDev& D, hipStream_t s);
// Each leaf's image of its LDS tables (after the tables, M fragments and Z values are current).
size_t panel_image_bytes(const PanelDev& D, int R, int prec, int warm);
hipError_t launch_panel_image(const PanelDev& D, const EmtDev& E, const HierDev& H, int R, int prec, int warm,
                              hipStream_t s);
hipError_t launch_emt_panel(const PanelDev& D, const EmtDev& E, const HierDev& H, const ModDev& M, const RunParams& P,
                            int prec, hipStream_t s);
// Level stepping (k_level.hip): LDS bytes of the layout, and the launch.
size_t level_lds_bytes(const LevelDev& D, int R, int prec, int warm);   // warm: FP64 incremental form
hipError_t launch_emt_level(const LevelDev& D, const EmtDev& E, const HierDev& H, const ModDev& M, const RunParams& P,
                            int prec, hipStream_t s);
// Several cases, each a team of its T workgroups, in as few cooperative launches as residency
// allows (d_cases: device table with wg0 the running sum of T; n_wg, sync: host arrays of each
// case's T and barrier flags; Ld: maxima of the LDS dimensions over the cases, R the largest rank).
hipError_t launch_emt_level_multi(const LevelDev& Ld, int R, const LevelCase* d_cases, const int* n_wg,
                                  unsigned int* const* sync, int n_cases, int n_steps, int prec, int warm,
                                  hipStream_t s);
// Fused stepping (k_run.hip): one workgroup per case, all steps in one launch.
bool run_fits(const HierDev& H);
size_t serve_lds_bytes(const HierDev& H, bool gvec);
hipError_t launch_emt_serve(const ServeSlot* d_slots, int n_slots, int n_steps, size_t lds, int prec, int warm,
                            hipStream_t s);
hipError_t launch_emt_run(const EmtDev& E, const HierDev& H, const ModDev& M, const RunParams& P, int prec,
                          hipStream_t s);
// History update with v_n and assembly of b_{n+1}; records; advances *E.step.
// New history of phase p of three-phase line l from the line's phase voltages v_ft and current
// histories: i = Y v_ft + h (3-vectors), h_p' = (Y v_ft)_p + (A i)_p.  One fixed operation order, so
// every caller (both ends of the line, every engine) gets the same bits.
__device__ inline double line3_history(const EmtDev& E, const double* v, const double* hcur, int l, int p)
{
    const double* Y = E.Y3 + 9 * l;
    const double* A = E.A3 + 9 * l;
    double vft[3], il[3];
    for (int r = 0; r < 3; ++r) vft[r] = v[E.fr[3 * l + r]] - v[E.to[3 * l + r]];
    double yv = 0.0;
    for (int r = 0; r < 3; ++r) {
        double y = 0.0;
        for (int c = 0; c < 3; ++c) y = fma(Y[3 * r + c], vft[c], y);
        il[r] = y + hcur[3 * l + r];
        if (r == p) yv = y;
    }
    double ai = 0.0;
    for (int c = 0; c < 3; ++c) ai = fma(A[3 * p + c], il[c], ai);
    return yv + ai;
}

void launch_emt_history(const EmtDev& E, const RecParams* rec, hipStream_t s);
// GMRES-based refinement (k_gmres.hip)
constexpr int kGmresMaxInner = 64;
void launch_gm_dots(int n, int nrhs, int nv, const double* V, const double* W, double sgn, double* out, int ld_out,
                    hipStream_t s);
void launch_gm_norms(int n, int nrhs, const double* W, double* out, hipStream_t s);
void launch_gm_update(int n, int nrhs, int nv, const double* V, const double* h, int ld_h, double sgn, double* W,
                      hipStream_t s);
void launch_gm_scale(int n, int nrhs, const double* W, const double* nrm, int ld_nrm, double sgn, double* Vout,
                     hipStream_t s);
void launch_gm_givens(int nrhs, int m, int j, const double* dots, const double* nrm, double* Hs, double* cs,
                      double* sn, double* g, double* res, hipStream_t s);
void launch_gm_start(int nrhs, int m, const double* nrm, double* g, double* res, hipStream_t s);
void launch_gm_backsolve(int nrhs, int m, int nj, const double* Hs, const double* g, double* y, hipStream_t s);
void launch_gm_jacobi(const HierDev& H, int nrhs, const double* R, double omega, double* Z, hipStream_t s);
void launch_emt_history3(const EmtDev& E, const RecParams* rec, hipStream_t s);

}  // namespace hinv
