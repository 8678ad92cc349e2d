// Host side of libhinv: argument validation, the partition-tree bookkeeping
// (bus renumbering, cut lines and their coupling columns, storage layout),
// workspace carving, and the C ABI declared in include/hinv.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cstring>

#include <algorithm>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hinv_internal.h"

using namespace hinv;

namespace {

thread_local std::string g_err;

hinv_status fail(hinv_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

}  // namespace

// The library's error string, for the other translation units.
hinv_status hinv::set_error(hinv_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

namespace {

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(HINV_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;

// Bump allocator over the caller's workspace; with base == nullptr it only measures.
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(int64_t count)
    {
        off = (off + kAlign - 1) / kAlign * kAlign;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += sizeof(T) * (size_t)(count > 0 ? count : 1);
        return p;
    }
};

int64_t align_elems(int64_t x) { return (x + 31) / 32 * 32; }

// ---------------------------------------------------------------------------
// Plan: everything about the hierarchy that depends only on G's pattern/values
// and the tree, computed on the host.
struct Plan {
    int n = 0, n_nodes = 0, n_levels = 0, anc_stride = 1;
    std::vector<int> perm, iperm;
    std::vector<int> leaf_lo, leaf_n, leaf_anc, row_leaf;
    std::vector<int64_t> leaf_off;
    std::vector<int> node_lo, node_n, node_m, node_col0, node_pan0, node_npan, node_level;
    std::vector<int64_t> node_soff;
    std::vector<int> pan_lo, pan_n, pan_col0, pan_m;
    std::vector<int64_t> pan_zoff;
    std::vector<int> col_row, col_partner, col_pan;
    std::vector<double> col_w, col_sign;
    std::vector<int> lvl_node, lvl_pan, lvl_col;
    std::vector<LevelHost> lv;
    std::vector<int> row_lo, row_nl, col_node, lvl_frow, frow_pan, pan_frow0;
    std::vector<int64_t> row_boff;
    std::vector<int> col_m, col_c0, frow_pn, frow_pm, frow_pc, frow_row;
    std::vector<int64_t> col_soff, frow_z;
    std::vector<int> rp, ci;
    std::vector<double> cv;
    int64_t leaf_entries = 0, z_entries = 0, s_entries = 0;
    int max_cols = 0, max_pan_rows = 0, max_leaf = 0;
    // capacitance inversions, level by level: gj_list[gj_at[h] .. gj_at[h] + gj_n[h]) are the
    // level's nodes with m > 0 in the order invert_level launches them
    std::vector<int> gj_list, gj_at, gj_n;
    int64_t gj_xb = 0, gj_sync = 0;   // exchange space of the largest team launch
};

// Order nodes for invert_level: m <= kNodeGjMax (one workgroup each), then m <= kGjTeamMax (a team
// of workgroups each), then the rest (one launch pair per pivot step).  Nodes with m == 0 drop out.
std::vector<int> order_nodes(const Plan& P, const std::vector<int>& nodes)
{
    std::vector<int> out;
    for (int pass = 0; pass < 3; ++pass)
        for (int t : nodes) {
            const int m = P.node_m[t];
            const int cat = m <= 0 ? -1 : m <= kNodeGjMax ? 0 : m <= kGjTeamMax ? 1 : 2;
            if (cat == pass) out.push_back(t);
        }
    return out;
}

hinv_status check_csr(const hinv_csr* G)
{
    if (!G) return fail(HINV_E_INVALID, "G is NULL");
    const int n = G->n;
    if (n < 1) return fail(HINV_E_INVALID, "n = %d < 1", n);
    if (!G->row_ptr || !G->col_idx || !G->val) return fail(HINV_E_INVALID, "CSR arrays must not be NULL");
    if (G->row_ptr[0] != 0) return fail(HINV_E_INVALID, "row_ptr[0] != 0");
    for (int i = 0; i < n; ++i) {
        if (G->row_ptr[i + 1] < G->row_ptr[i]) return fail(HINV_E_INVALID, "row_ptr not non-decreasing at %d", i);
        bool diag = false;
        for (int e = G->row_ptr[i]; e < G->row_ptr[i + 1]; ++e) {
            const int c = G->col_idx[e];
            if (c < 0 || c >= n) return fail(HINV_E_INVALID, "column index %d out of range in row %d", c, i);
            if (e > G->row_ptr[i] && G->col_idx[e - 1] >= c)
                return fail(HINV_E_INVALID, "columns of row %d not strictly increasing", i);
            if (!isfinite(G->val[e])) return fail(HINV_E_INVALID, "non-finite value in row %d", i);
            if (c == i) {
                diag = true;
                if (!(G->val[e] > 0.0)) return fail(HINV_E_NOT_SPD, "diagonal G[%d][%d] = %g is not positive", i, i, G->val[e]);
            } else {
                const int* b = G->col_idx + G->row_ptr[c];
                const int* en = G->col_idx + G->row_ptr[c + 1];
                const int* f = std::lower_bound(b, en, i);
                if (f == en || *f != i) return fail(HINV_E_INVALID, "G is not symmetric: (%d,%d) has no mirror", i, c);
                if (G->val[G->row_ptr[c] + (f - b)] != G->val[e])
                    return fail(HINV_E_INVALID, "G is not symmetric: G[%d][%d] != G[%d][%d]", i, c, c, i);
            }
        }
        if (!diag) return fail(HINV_E_INVALID, "row %d has no diagonal entry", i);
    }
    return HINV_OK;
}

}  // namespace

hinv_status hinv::validate_csr(const hinv_csr* G) { return check_csr(G); }

namespace {

hinv_status make_plan(const hinv_csr* G, const hinv_tree* T, Plan& P)
{
    hinv_status st = check_csr(G);
    if (st != HINV_OK) return st;
    if (!T || !T->parent || !T->bus_leaf || T->n_nodes < 1) return fail(HINV_E_INVALID, "tree is missing or empty");
    const int n = G->n, nn = T->n_nodes;
    P.n = n;
    P.n_nodes = nn;
    std::vector<std::vector<int>> children(nn);
    int root = -1;
    for (int k = 0; k < nn; ++k) {
        const int p = T->parent[k];
        if (p == -1) {
            if (root >= 0) return fail(HINV_E_INVALID, "tree has two roots (%d and %d)", root, k);
            root = k;
        } else if (p < 0 || p >= nn || p == k) {
            return fail(HINV_E_INVALID, "parent[%d] = %d is invalid", k, p);
        } else {
            children[p].push_back(k);
        }
    }
    if (root < 0) return fail(HINV_E_INVALID, "tree has no root");
    std::vector<int> depth(nn, -1);
    // depth by walking up (bounded: a cycle never reaches the root)
    for (int k = 0; k < nn; ++k) {
        int d = 0, x = k;
        while (x != root) {
            x = T->parent[x];
            if (++d > nn) return fail(HINV_E_INVALID, "tree has a cycle through node %d", k);
        }
        depth[k] = d;
    }
    std::vector<std::vector<int>> leaf_buses(nn);
    for (int a = 0; a < n; ++a) {
        const int l = T->bus_leaf[a];
        if (l < 0 || l >= nn) return fail(HINV_E_INVALID, "bus_leaf[%d] = %d out of range", a, l);
        if (!children[l].empty()) return fail(HINV_E_INVALID, "bus %d is assigned to internal node %d", a, l);
        leaf_buses[l].push_back(a);
    }
    // depth-first order (children in index order); post-order for ranges and heights
    std::vector<int> order, stack{root};
    std::vector<int> leaf_of_node(nn, -1);
    while (!stack.empty()) {
        const int x = stack.back();
        stack.pop_back();
        order.push_back(x);
        for (int i = (int)children[x].size() - 1; i >= 0; --i) stack.push_back(children[x][i]);
    }
    std::vector<int> lo(nn, 0), hi(nn, 0), height(nn, 0);
    P.perm.clear();
    for (int x : order) {
        if (children[x].empty()) {
            if (leaf_buses[x].empty()) return fail(HINV_E_INVALID, "leaf %d owns no bus", x);
            if ((int)leaf_buses[x].size() > kMaxLeaf)
                return fail(HINV_E_INVALID, "leaf %d owns %d buses (limit %d)", x, (int)leaf_buses[x].size(), kMaxLeaf);
            leaf_of_node[x] = (int)P.leaf_lo.size();
            lo[x] = (int)P.perm.size();
            for (int a : leaf_buses[x]) P.perm.push_back(a);
            hi[x] = (int)P.perm.size();
            P.leaf_lo.push_back(lo[x]);
            P.leaf_n.push_back(hi[x] - lo[x]);
        }
    }
    if ((int)P.perm.size() != n) return fail(HINV_E_INVALID, "tree leaves do not cover all buses");
    for (int i = (int)order.size() - 1; i >= 0; --i) {
        const int x = order[i];
        if (children[x].empty()) continue;
        lo[x] = lo[children[x].front()];
        hi[x] = hi[children[x].back()];
        int h = 0;
        for (int c : children[x]) h = std::max(h, height[c] + 1);
        height[x] = h;
    }
    P.iperm.assign(n, 0);
    for (int r = 0; r < n; ++r) P.iperm[P.perm[r]] = r;
    P.n_levels = height[root];
    // internal nodes ordered by (height, id)
    std::vector<int> internal;
    for (int k = 0; k < nn; ++k)
        if (!children[k].empty()) internal.push_back(k);
    std::stable_sort(internal.begin(), internal.end(), [&](int x, int y) { return height[x] < height[y]; });
    std::vector<int> int_idx(nn, -1);
    for (size_t i = 0; i < internal.size(); ++i) int_idx[internal[i]] = (int)i;
    // leaves: offsets, ancestors, row -> leaf
    const int L = (int)P.leaf_lo.size();
    int maxdepth = 1;
    for (int k = 0; k < nn; ++k) maxdepth = std::max(maxdepth, depth[k]);
    P.anc_stride = maxdepth;
    P.leaf_anc.assign((size_t)L * maxdepth, -1);
    P.row_leaf.assign(n, 0);
    P.leaf_off.resize(L);
    int64_t off = 0;
    for (int x : order) {
        const int l = leaf_of_node[x];
        if (l < 0) continue;
        P.leaf_off[l] = off;
        off += align_elems((int64_t)P.leaf_n[l] * P.leaf_n[l]);
        P.max_leaf = std::max(P.max_leaf, P.leaf_n[l]);
        for (int r = P.leaf_lo[l]; r < P.leaf_lo[l] + P.leaf_n[l]; ++r) P.row_leaf[r] = l;
        int y = x, d = 0;
        while (y != root) {
            y = T->parent[y];
            P.leaf_anc[(size_t)l * maxdepth + d++] = int_idx[y];
        }
    }
    P.leaf_entries = off;
    // node of each leaf index (tree node id)
    std::vector<int> leaf_node(L);
    for (int k = 0; k < nn; ++k)
        if (leaf_of_node[k] >= 0) leaf_node[leaf_of_node[k]] = k;
    // permuted CSR
    P.rp.assign(n + 1, 0);
    for (int r = 0; r < n; ++r) {
        const int a = P.perm[r];
        P.rp[r + 1] = P.rp[r] + (G->row_ptr[a + 1] - G->row_ptr[a]);
    }
    P.ci.resize(P.rp[n]);
    P.cv.resize(P.rp[n]);
    {
        std::vector<std::pair<int, double>> row;
        for (int r = 0; r < n; ++r) {
            const int a = P.perm[r];
            row.clear();
            for (int e = G->row_ptr[a]; e < G->row_ptr[a + 1]; ++e) row.push_back({P.iperm[G->col_idx[e]], G->val[e]});
            std::sort(row.begin(), row.end(), [](const std::pair<int, double>& x, const std::pair<int, double>& y) {
                return x.first < y.first;
            });
            for (size_t q = 0; q < row.size(); ++q) {
                P.ci[P.rp[r] + q] = row[q].first;
                P.cv[P.rp[r] + q] = row[q].second;
            }
        }
    }
    // cut lines: entry (r, c), r < c, in different leaves, belongs to their lowest common ancestor
    struct Cut { int r, c, cr, cc; double val; };
    std::vector<std::vector<Cut>> cuts(internal.size());
    for (int r = 0; r < n; ++r) {
        for (int e = P.rp[r]; e < P.rp[r + 1]; ++e) {
            const int c = P.ci[e];
            if (c <= r || P.cv[e] == 0.0) continue;
            int x = leaf_node[P.row_leaf[r]], y = leaf_node[P.row_leaf[c]];
            if (x == y) continue;
            int px = -1, py = -1;
            while (depth[x] > depth[y]) { px = x; x = T->parent[x]; }
            while (depth[y] > depth[x]) { py = y; y = T->parent[y]; }
            while (x != y) { px = x; x = T->parent[x]; py = y; y = T->parent[y]; }
            cuts[int_idx[x]].push_back({r, c, px, py, P.cv[e]});
        }
    }
    // columns and panels, node by node in level order
    const int NI = (int)internal.size();
    P.node_lo.resize(NI); P.node_n.resize(NI); P.node_m.resize(NI); P.node_col0.resize(NI);
    P.node_pan0.resize(NI); P.node_npan.resize(NI); P.node_level.resize(NI); P.node_soff.resize(NI);
    P.lvl_node.assign(P.n_levels + 1, 0);
    P.lvl_pan.assign(P.n_levels + 1, 0);
    P.lvl_col.assign(P.n_levels + 1, 0);
    P.lv.assign(P.n_levels, LevelHost{0, 0, 0, 0, 0});
    int64_t soff = 0, zoff = 0;
    for (int i = 0; i < NI; ++i) {
        const int t = internal[i];
        const int h = height[t];
        P.node_lo[i] = lo[t];
        P.node_n[i] = hi[t] - lo[t];
        P.node_level[i] = h;
        P.node_col0[i] = (int)P.col_row.size();
        P.node_pan0[i] = (int)P.pan_lo.size();
        const std::vector<Cut>& cs = cuts[i];
        const int m = 2 * (int)cs.size();
        P.node_m[i] = m;
        P.node_soff[i] = soff;
        soff += align_elems((int64_t)m * m);
        // endpoint columns grouped by child
        std::vector<int> col_of_end(2 * cs.size(), -1);
        for (int c : children[t]) {
            const int pan = (int)P.pan_lo.size();
            const int col0 = (int)P.col_row.size();
            for (size_t j = 0; j < cs.size(); ++j) {
                if (cs[j].cr == c) { col_of_end[2 * j] = (int)P.col_row.size(); P.col_row.push_back(cs[j].r); }
                if (cs[j].cc == c) { col_of_end[2 * j + 1] = (int)P.col_row.size(); P.col_row.push_back(cs[j].c); }
            }
            const int pm = (int)P.col_row.size() - col0;
            if (pm == 0) continue;
            P.pan_lo.push_back(lo[c]);
            P.pan_n.push_back(hi[c] - lo[c]);
            P.pan_col0.push_back(col0);
            P.pan_m.push_back(pm);
            P.pan_zoff.push_back(zoff);
            zoff += align_elems((int64_t)(hi[c] - lo[c]) * pm);
            for (int q = 0; q < pm; ++q) P.col_pan.push_back(pan);
            P.max_pan_rows = std::max(P.max_pan_rows, hi[c] - lo[c]);
            P.lv[h - 1].max_pan_rows = std::max(P.lv[h - 1].max_pan_rows, hi[c] - lo[c]);
        }
        P.col_w.resize(P.col_row.size());
        P.col_sign.resize(P.col_row.size());
        P.col_partner.resize(P.col_row.size());
        for (size_t j = 0; j < cs.size(); ++j) {
            const int ca = col_of_end[2 * j], cb = col_of_end[2 * j + 1];
            const double w = sqrt(fabs(cs[j].val)), sg = cs[j].val > 0 ? 1.0 : -1.0;
            P.col_w[ca] = w; P.col_w[cb] = w;
            P.col_sign[ca] = sg; P.col_sign[cb] = sg;
            P.col_partner[ca] = cb; P.col_partner[cb] = ca;
        }
        P.node_npan[i] = (int)P.pan_lo.size() - P.node_pan0[i];
        P.max_cols = std::max(P.max_cols, m);
        LevelHost& Lh = P.lv[h - 1];
        Lh.nnodes += 1;
        Lh.npan += P.node_npan[i];
        Lh.ncols += m;
        Lh.max_m = std::max(Lh.max_m, m);
        P.lvl_node[h] = i + 1;
        P.lvl_pan[h] = (int)P.pan_lo.size();
        P.lvl_col[h] = (int)P.col_row.size();
    }
    for (int h = 1; h <= P.n_levels; ++h) {   // empty levels inherit the previous end
        if (P.lvl_node[h] < P.lvl_node[h - 1]) P.lvl_node[h] = P.lvl_node[h - 1];
        if (P.lvl_pan[h] < P.lvl_pan[h - 1]) P.lvl_pan[h] = P.lvl_pan[h - 1];
        if (P.lvl_col[h] < P.lvl_col[h - 1]) P.lvl_col[h] = P.lvl_col[h - 1];
    }
    P.z_entries = zoff;
    P.s_entries = soff;
    // lookups for the fused kernel
    P.row_lo.resize(n); P.row_nl.resize(n); P.row_boff.resize(n);
    for (int r = 0; r < n; ++r) {
        const int l = P.row_leaf[r];
        P.row_lo[r] = P.leaf_lo[l];
        P.row_nl[r] = P.leaf_n[l];
        P.row_boff[r] = P.leaf_off[l] + (r - P.leaf_lo[l]);
    }
    P.col_node.resize(P.col_row.size());
    for (int i = 0; i < NI; ++i)
        for (int q = 0; q < P.node_m[i]; ++q) P.col_node[P.node_col0[i] + q] = i;
    P.lvl_frow.assign(P.n_levels + 1, 0);
    P.pan_frow0.resize(P.pan_lo.size());
    for (int h = 1; h <= P.n_levels; ++h) {
        for (int pp = P.lvl_pan[h - 1]; pp < P.lvl_pan[h]; ++pp) {
            P.pan_frow0[pp] = (int)P.frow_pan.size();
            for (int i = 0; i < P.pan_n[pp]; ++i) {
                P.frow_pan.push_back(pp);
                P.frow_z.push_back(P.pan_zoff[pp] + i);
                P.frow_pn.push_back(P.pan_n[pp]);
                P.frow_pm.push_back(P.pan_m[pp]);
                P.frow_pc.push_back(P.pan_col0[pp]);
                P.frow_row.push_back(P.pan_lo[pp] + i);
            }
        }
        P.lvl_frow[h] = (int)P.frow_pan.size();
    }
    P.col_m.resize(P.col_row.size()); P.col_c0.resize(P.col_row.size()); P.col_soff.resize(P.col_row.size());
    for (size_t g = 0; g < P.col_row.size(); ++g) {
        const int t = P.col_node[g];
        P.col_m[g] = P.node_m[t];
        P.col_c0[g] = P.node_col0[t];
        P.col_soff[g] = P.node_soff[t] + ((int)g - P.node_col0[t]);
    }
    if (P.max_cols > 4096) return fail(HINV_E_INVALID, "a tree node has %d coupling columns (limit 4096)", P.max_cols);
    P.gj_at.assign(P.n_levels + 1, 0);
    P.gj_n.assign(P.n_levels + 1, 0);
    for (int h = 1; h <= P.n_levels; ++h) {
        std::vector<int> lvl;
        for (int t = P.lvl_node[h - 1]; t < P.lvl_node[h]; ++t) lvl.push_back(t);
        const std::vector<int> ord = order_nodes(P, lvl);
        P.gj_at[h] = (int)P.gj_list.size();
        P.gj_n[h] = (int)ord.size();
        P.gj_list.insert(P.gj_list.end(), ord.begin(), ord.end());
        std::vector<int> mt;
        for (int t : ord)
            if (P.node_m[t] > kNodeGjMax && P.node_m[t] <= kGjTeamMax) mt.push_back(P.node_m[t]);
        int64_t xbd = 0, syw = 0;
        gj_team_sizes(mt, &xbd, &syw);
        P.gj_xb = std::max(P.gj_xb, xbd);
        P.gj_sync = std::max(P.gj_sync, syw);
    }
    return HINV_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
struct hinv_ctx {
    Plan P;
    hinv_options opt{};
    HierDev H{};
    ModDev M{};            // one change set (hinv_modify_line)
    int* d_perm = nullptr;
    int* d_flags = nullptr;
    double* colbuf = nullptr;
    int* ipiv = nullptr;
    double *X = nullptr, *Xo = nullptr, *D = nullptr, *Rv = nullptr, *Y = nullptr;
    unsigned long long* stats = nullptr;
    // change-set host mirror
    std::vector<int> mod_a, mod_b, mod_act;
    std::vector<double> mod_dg;
    int* m_count = nullptr; int* m_a = nullptr; int* m_b = nullptr; int* m_act = nullptr; double* m_dg = nullptr;
    int* upd_list = nullptr;   // leaves / columns / nodes a local rebuild launches over
    int* gj_list = nullptr;    // the plan's per-level capacitance inversion lists
    double* gj_xb = nullptr;   // team Gauss-Jordan exchange
    unsigned int* gj_sync = nullptr;
    int64_t applies = 0;
};

namespace {

// Carve the hierarchy's device storage (base == nullptr: measure only).
void carve_hier(hinv_ctx& c, Arena& A, int n_sets, int R, int max_nrhs)
{
    const Plan& P = c.P;
    HierDev& H = c.H;
    const int L = (int)P.leaf_lo.size(), NI = (int)P.node_lo.size(), NP = (int)P.pan_lo.size();
    const int NC = (int)P.col_row.size();
    H.n = P.n; H.n_leaves = L; H.n_internal = NI; H.n_levels = P.n_levels; H.n_cols = NC;
    H.anc_stride = P.anc_stride; H.max_cols = P.max_cols; H.max_pan_rows = P.max_pan_rows;
    c.d_perm = A.take<int>(P.n);
    H.leaf_lo = A.take<int>(L); H.leaf_n = A.take<int>(L); H.leaf_off = A.take<int64_t>(L);
    H.leaf_anc = A.take<int>((int64_t)L * P.anc_stride); H.row_leaf = A.take<int>(P.n);
    H.node_lo = A.take<int>(NI); H.node_n = A.take<int>(NI); H.node_m = A.take<int>(NI);
    H.node_col0 = A.take<int>(NI); H.node_soff = A.take<int64_t>(NI); H.node_pan0 = A.take<int>(NI);
    H.node_npan = A.take<int>(NI); H.node_level = A.take<int>(NI);
    H.pan_lo = A.take<int>(NP); H.pan_n = A.take<int>(NP); H.pan_col0 = A.take<int>(NP); H.pan_m = A.take<int>(NP);
    H.pan_zoff = A.take<int64_t>(NP);
    H.col_row = A.take<int>(NC); H.col_w = A.take<double>(NC); H.col_partner = A.take<int>(NC);
    H.col_sign = A.take<double>(NC); H.col_pan = A.take<int>(NC);
    H.lvl_node = A.take<int>(P.n_levels + 1); H.lvl_pan = A.take<int>(P.n_levels + 1);
    H.lvl_col = A.take<int>(P.n_levels + 1);
    H.row_lo = A.take<int>(P.n); H.row_nl = A.take<int>(P.n); H.row_boff = A.take<int64_t>(P.n);
    H.col_node = A.take<int>(NC); H.lvl_frow = A.take<int>(P.n_levels + 1);
    H.frow_pan = A.take<int>((int64_t)P.frow_pan.size()); H.pan_frow0 = A.take<int>(NP);
    H.col_m = A.take<int>(NC); H.col_c0 = A.take<int>(NC); H.col_soff = A.take<int64_t>(NC);
    {
        const int64_t nf = (int64_t)P.frow_pan.size();
        H.frow_z = A.take<int64_t>(nf); H.frow_pn = A.take<int>(nf); H.frow_pm = A.take<int>(nf);
        H.frow_pc = A.take<int>(nf); H.frow_row = A.take<int>(nf);
    }
    H.rp = A.take<int>(P.n + 1); H.ci = A.take<int>(P.rp.empty() ? 1 : P.rp[P.n]);
    H.cv = A.take<double>(P.rp.empty() ? 1 : P.rp[P.n]);
    H.blk = A.take<double>(P.leaf_entries); H.Z = A.take<double>(P.z_entries); H.Sinv = A.take<double>(P.s_entries);
    H.blk32 = H.Z32 = H.Sinv32 = nullptr;
    H.blk16 = H.Z16 = H.Sinv16 = nullptr;
    H.blk8 = H.Z8 = H.Sinv8 = H.blk8s = H.Z8s = H.Sinv8s = nullptr;
    if (c.opt.prec == HINV_FP32) {
        H.blk32 = A.take<float>(P.leaf_entries); H.Z32 = A.take<float>(P.z_entries);
        H.Sinv32 = A.take<float>(P.s_entries);
    } else if (c.opt.prec == HINV_BF16) {
        H.blk16 = A.take<uint16_t>(P.leaf_entries); H.Z16 = A.take<uint16_t>(P.z_entries);
        H.Sinv16 = A.take<uint16_t>(P.s_entries);
    } else if (c.opt.prec == HINV_FP8) {
        H.blk8 = A.take<uint8_t>(P.leaf_entries); H.Z8 = A.take<uint8_t>(P.z_entries);
        H.Sinv8 = A.take<uint8_t>(P.s_entries);
        H.blk8s = A.take<uint8_t>(P.leaf_entries / 32 + 1); H.Z8s = A.take<uint8_t>(P.z_entries / 32 + 1);
        H.Sinv8s = A.take<uint8_t>(P.s_entries / 32 + 1);
    }
    c.colbuf = A.take<double>(NC);
    c.ipiv = A.take<int>(NC);
    c.upd_list = A.take<int>((int64_t)L + NC + NI);
    c.gj_list = A.take<int>(NI);
    c.gj_xb = A.take<double>(P.gj_xb);
    c.gj_sync = A.take<unsigned int>(P.gj_sync);
    c.d_flags = A.take<int>(4);
    c.X = A.take<double>((int64_t)P.n * max_nrhs);
    c.Xo = A.take<double>((int64_t)P.n * max_nrhs);
    c.D = A.take<double>((int64_t)P.n * max_nrhs);
    c.Rv = A.take<double>((int64_t)P.n * max_nrhs);
    c.Y = A.take<double>((int64_t)NC * max_nrhs);
    c.stats = A.take<unsigned long long>((int64_t)max_nrhs);
    // change sets
    ModDev& M = c.M;
    M.n_sets = n_sets; M.R = R; M.n = P.n;
    c.m_count = A.take<int>(n_sets);
    c.m_a = A.take<int>((int64_t)n_sets * R); c.m_b = A.take<int>((int64_t)n_sets * R);
    c.m_act = A.take<int>((int64_t)n_sets * R); c.m_dg = A.take<double>((int64_t)n_sets * R);
    M.count = c.m_count; M.a = c.m_a; M.b = c.m_b; M.act = c.m_act; M.dg = c.m_dg;
    M.U = A.take<double>((int64_t)n_sets * R * P.n);
    M.U32 = (c.opt.prec != HINV_FP64) ? A.take<float>((int64_t)n_sets * R * P.n) : nullptr;
    M.Cinv = A.take<double>((int64_t)n_sets * R * R * R);
}

template <typename T>
hipError_t up(const T* dst, const std::vector<T>& src, hipStream_t s)
{
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync((void*)dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s);
}

hinv_status check_options(const hinv_options* o, int min_nrhs)
{
    if (!o) return fail(HINV_E_INVALID, "options are NULL");
    if (o->prec < HINV_FP64 || o->prec > HINV_FP8) return fail(HINV_E_INVALID, "unknown precision %d", o->prec);
    if (o->max_mod_rank < 0 || o->max_mod_rank > kMaxModRank)
        return fail(HINV_E_INVALID, "max_mod_rank %d outside 0..%d", o->max_mod_rank, kMaxModRank);
    if (o->max_nrhs < min_nrhs) return fail(HINV_E_INVALID, "max_nrhs %d < %d", o->max_nrhs, min_nrhs);
    if (o->coupling != HINV_COUPLING_EXACT && o->coupling != HINV_COUPLING_PAPER)
        return fail(HINV_E_INVALID, "coupling %d unknown", o->coupling);
    const bool refines = o->prec != HINV_FP64 || o->coupling == HINV_COUPLING_PAPER;
    if (refines && (o->max_refine < 0 || o->max_refine > 64))
        return fail(HINV_E_INVALID, "max_refine %d outside 0..64", o->max_refine);
    if (o->kernel_mode < 0 || o->kernel_mode > 5) return fail(HINV_E_INVALID, "kernel_mode %d unknown", o->kernel_mode);
    if (refines && !(o->rel_tol >= 0.0)) return fail(HINV_E_INVALID, "rel_tol must be >= 0");
    return HINV_OK;
}

// Low-precision copies of the FP64 blocks, panels and capacitance inverses.
void convert_low(hinv_ctx& c, hipStream_t s)
{
    const Plan& P = c.P;
    HierDev& H = c.H;
    if (c.opt.prec == HINV_FP32) {
        launch_to_f32(H.blk, H.blk32, P.leaf_entries, s);
        launch_to_f32(H.Z, H.Z32, P.z_entries, s);
        launch_to_f32(H.Sinv, H.Sinv32, P.s_entries, s);
    } else if (c.opt.prec == HINV_BF16) {
        launch_to_bf16(H.blk, H.blk16, P.leaf_entries, s);
        launch_to_bf16(H.Z, H.Z16, P.z_entries, s);
        launch_to_bf16(H.Sinv, H.Sinv16, P.s_entries, s);
    } else if (c.opt.prec == HINV_FP8) {
        launch_to_fp8(H.blk, H.blk8, H.blk8s, P.leaf_entries, s);
        launch_to_fp8(H.Z, H.Z8, H.Z8s, P.z_entries, s);
        launch_to_fp8(H.Sinv, H.Sinv8, H.Sinv8s, P.s_entries, s);
    }
}

// S^{-1} of the nodes of one level: d_list (device) and nodes (host) hold the same nodes in
// order_nodes order.
hinv_status invert_level(hinv_ctx& c, int level, const int* d_list, const std::vector<int>& nodes, hipStream_t s)
{
    const Plan& P = c.P;
    int ns = 0, nl = 0, ml = 0;
    std::vector<int> mt;
    for (int t : nodes) {
        const int m = P.node_m[t];
        if (m <= kNodeGjMax) ++ns;
        else if (m <= kGjTeamMax) mt.push_back(m);
        else { ++nl; ml = std::max(ml, m); }
    }
    const int nt = (int)mt.size();
    if (c.opt.coupling == HINV_COUPLING_PAPER) {      // Algorithm 1 as printed: S^{-1} := C (C^{-1} = C)
        int m_max = 0;
        for (int t : nodes) m_max = std::max(m_max, P.node_m[t]);
        launch_fill_s(c.H, level, (int)nodes.size(), m_max, s, d_list, /*coupling_only=*/true);
        return HINV_OK;
    }
    launch_node_inverse(c.H, d_list, ns, c.d_flags, s);
    HIP_TRY(launch_gj_team(c.H, d_list + ns, mt, c.gj_xb, c.gj_sync, c.d_flags, s));
    if (nl > 0) {
        const int* lst = d_list + ns + nt;
        launch_fill_s(c.H, level, nl, ml, s, lst);
        launch_gj_level(c.H, level, nl, ml, c.colbuf, c.ipiv, c.d_flags, s, lst);
    }
    return HINV_OK;
}

// Upload the plan and run the FP64 build (leaf inverses, then per level Z and S^{-1}).
hinv_status build_device(hinv_ctx& c, hipStream_t s)
{
    const Plan& P = c.P;
    HierDev& H = c.H;
    HIP_TRY(up(c.d_perm, P.perm, s));
    HIP_TRY(up(H.leaf_lo, P.leaf_lo, s)); HIP_TRY(up(H.leaf_n, P.leaf_n, s)); HIP_TRY(up(H.leaf_off, P.leaf_off, s));
    HIP_TRY(up(H.leaf_anc, P.leaf_anc, s)); HIP_TRY(up(H.row_leaf, P.row_leaf, s));
    HIP_TRY(up(H.node_lo, P.node_lo, s)); HIP_TRY(up(H.node_n, P.node_n, s)); HIP_TRY(up(H.node_m, P.node_m, s));
    HIP_TRY(up(H.node_col0, P.node_col0, s)); HIP_TRY(up(H.node_soff, P.node_soff, s));
    HIP_TRY(up(H.node_pan0, P.node_pan0, s)); HIP_TRY(up(H.node_npan, P.node_npan, s));
    HIP_TRY(up(H.node_level, P.node_level, s));
    HIP_TRY(up(H.pan_lo, P.pan_lo, s)); HIP_TRY(up(H.pan_n, P.pan_n, s)); HIP_TRY(up(H.pan_col0, P.pan_col0, s));
    HIP_TRY(up(H.pan_m, P.pan_m, s)); HIP_TRY(up(H.pan_zoff, P.pan_zoff, s));
    HIP_TRY(up(H.col_row, P.col_row, s)); HIP_TRY(up(H.col_w, P.col_w, s)); HIP_TRY(up(H.col_partner, P.col_partner, s));
    HIP_TRY(up(H.col_sign, P.col_sign, s)); HIP_TRY(up(H.col_pan, P.col_pan, s));
    HIP_TRY(up(H.lvl_node, P.lvl_node, s)); HIP_TRY(up(H.lvl_pan, P.lvl_pan, s)); HIP_TRY(up(H.lvl_col, P.lvl_col, s));
    HIP_TRY(up(H.row_lo, P.row_lo, s)); HIP_TRY(up(H.row_nl, P.row_nl, s)); HIP_TRY(up(H.row_boff, P.row_boff, s));
    HIP_TRY(up(H.col_node, P.col_node, s)); HIP_TRY(up(H.lvl_frow, P.lvl_frow, s));
    HIP_TRY(up(H.frow_pan, P.frow_pan, s)); HIP_TRY(up(H.pan_frow0, P.pan_frow0, s));
    HIP_TRY(up(H.col_m, P.col_m, s)); HIP_TRY(up(H.col_c0, P.col_c0, s)); HIP_TRY(up(H.col_soff, P.col_soff, s));
    HIP_TRY(up(H.frow_z, P.frow_z, s)); HIP_TRY(up(H.frow_pn, P.frow_pn, s)); HIP_TRY(up(H.frow_pm, P.frow_pm, s));
    HIP_TRY(up(H.frow_pc, P.frow_pc, s)); HIP_TRY(up(H.frow_row, P.frow_row, s));
    HIP_TRY(up(H.rp, P.rp, s)); HIP_TRY(up(H.ci, P.ci, s)); HIP_TRY(up(H.cv, P.cv, s));
    HIP_TRY(up(c.gj_list, P.gj_list, s));
    HIP_TRY(hipMemsetAsync(c.d_flags, 0, 4 * sizeof(int), s));
    HIP_TRY(hipMemsetAsync((void*)c.M.count, 0, sizeof(int) * c.M.n_sets, s));
    HIP_TRY(hipMemsetAsync(c.stats, 0, sizeof(unsigned long long) * c.opt.max_nrhs, s));
    launch_leaf_inverse(H, c.d_flags, s);
    for (int l = 1; l <= P.n_levels; ++l) {
        const LevelHost& L = P.lv[l - 1];
        if (L.nnodes == 0 || L.ncols == 0) continue;
        launch_build_z(H, l, L.ncols, s);
        const std::vector<int> nodes(P.gj_list.begin() + P.gj_at[l], P.gj_list.begin() + P.gj_at[l] + P.gj_n[l]);
        hinv_status st = invert_level(c, l, c.gj_list + P.gj_at[l], nodes, s);
        if (st != HINV_OK) return st;
    }
    convert_low(c, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    int flags = 0;
    HIP_TRY(hipMemcpy(&flags, c.d_flags, sizeof(int), hipMemcpyDeviceToHost));
    if (flags & kFlagNotSPD) return fail(HINV_E_NOT_SPD, "a leaf block of G is not positive definite");
    if (flags & kFlagSingular) return fail(HINV_E_SINGULAR, "a coupling capacitance matrix is singular");
    if (flags & kFlagBarrier) return fail(HINV_E_DEVICE, "a workgroup team of the build timed out at a barrier");
    return HINV_OK;
}

// v = P x for nrhs columns already in the new order (X -> out), in the apply
// precision, including the active line changes of sets set0.. .
// Per-call temporaries of a solve: level values Y [nrhs * n_cols], residual Rv and correction D
// [nrhs * n], per-column convergence stats [nrhs].
struct SolveTemps {
    double* Y;
    double* Rv;
    double* D;
    unsigned long long* stats;
};

void precond(hinv_ctx& c, const SolveTemps& w, int prec, const double* X, double* out, int nrhs, int set_stride,
             const int64_t* step, hipStream_t s)
{
    launch_apply(c.H, c.P.lv.data(), prec, X, out, w.Y, nrhs, s);
    launch_smw_apply(c.M, prec, out, nrhs, 0, set_stride, step, s);
}

// Full solve in the new order: FP64 apply, or low-precision apply + FP64
// refinement.  set_stride 0: every column uses change set 0; 1: column k uses set k.
void solve_new_order(hinv_ctx& c, const SolveTemps& w, const double* B, double* V, int nrhs, int set_stride,
                     const int64_t* step, hipStream_t s)
{
    if (c.opt.prec == HINV_FP64 && c.opt.coupling == HINV_COUPLING_EXACT) {
        precond(c, w, HINV_FP64, B, V, nrhs, set_stride, step, s);
        c.applies += nrhs;
        return;
    }
    precond(c, w, c.opt.prec, B, V, nrhs, set_stride, step, s);
    for (int it = 0; it < c.opt.max_refine; ++it) {
        launch_residual(c.H, c.M, B, V, w.Rv, nrhs, set_stride, step, s);
        precond(c, w, c.opt.prec, w.Rv, w.D, nrhs, set_stride, step, s);
        launch_axpy_stats(c.P.n, nrhs, V, w.D, (it == c.opt.max_refine - 1) ? w.stats : nullptr, c.opt.rel_tol,
                          c.d_flags, s);
    }
    c.applies += (int64_t)nrhs * (1 + c.opt.max_refine);
}

// the same with the temporaries of the handle's own workspace
void solve_new_order(hinv_ctx& c, const double* B, double* V, int nrhs, int set_stride, const int64_t* step,
                     hipStream_t s)
{
    solve_new_order(c, SolveTemps{c.Y, c.Rv, c.D, c.stats}, B, V, nrhs, set_stride, step, s);
}

// Solve that starts from the previous solution in V (EMT with warm_start): passes of v += P (b - G v).
// FP64 storage: one pass, the incremental form.  Through a unit eigenvalue of the companion update
// (a floating bus) P b alone carries P's rounding forward from step to step; the residual form keeps
// each step's error at one apply's rounding of the step's change.  Lower storage precisions:
// max_refine + 1 passes, the last one's ||d|| / ||v|| checked against rel_tol.  Handle's own
// temporaries; V holds zeros before the first step.
void solve_from_previous(hinv_ctx& c, const double* B, double* V, int nrhs, int set_stride, const int64_t* step,
                         hipStream_t s)
{
    const SolveTemps w{c.Y, c.Rv, c.D, c.stats};
    const bool fp64 = c.opt.prec == HINV_FP64;
    const int passes = fp64 ? 1 : c.opt.max_refine + 1;
    for (int it = 0; it < passes; ++it) {
        launch_residual(c.H, c.M, B, V, w.Rv, nrhs, set_stride, step, s);
        precond(c, w, c.opt.prec, w.Rv, w.D, nrhs, set_stride, step, s);
        const bool last = !fp64 && it == passes - 1;
        launch_axpy_stats(c.P.n, nrhs, V, w.D, last ? w.stats : nullptr, last ? c.opt.rel_tol : 1e300, c.d_flags, s);
    }
    c.applies += (int64_t)nrhs * passes;
}

// Stored change j of set 0: u_j = G0^{-1} (e_a - e_b) by one FP64 apply of the current hierarchy.
hinv_status store_mod_u(hinv_ctx& c, int j, hipStream_t s)
{
    const int n = c.P.n;
    std::vector<double> w(n, 0.0);
    w[c.mod_a[j]] = 1.0;
    if (c.mod_b[j] >= 0) w[c.mod_b[j]] = -1.0;
    HIP_TRY(hipMemcpyAsync(c.X, w.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    launch_apply(c.H, c.P.lv.data(), HINV_FP64, c.X, c.Xo, c.Y, 1, s);
    HIP_TRY(hipMemcpyAsync(c.M.U + (int64_t)j * n, c.Xo, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if (c.M.U32) launch_to_f32(c.M.U + (int64_t)j * n, c.M.U32 + (int64_t)j * n, n, s);
    HIP_TRY(hipStreamSynchronize(s));   // w is pageable and local
    return HINV_OK;
}

// What a change of G inside leaves la, lb (and of the coupling column pair of a line between them)
// reaches in the stored inverse (Section IV, Algorithm 2, made exact): the two leaf blocks; at every
// ancestor of the two leaves, the panels Z of the children that contain one of them (their subtree
// matrix changed, or for the line's own pair at the lowest common ancestor its weight) and, where a
// panel changed, the capacitance inverse.  Ancestors above the lowest common ancestor are included:
// their children's subtree matrices changed too, so stopping there would leave the inverse
// approximate.  Everything else keeps inputs identical to a full build.
struct LocalSet {
    std::vector<int> leaves;
    std::vector<std::vector<int>> cols, nodes;   // per level 1..n_levels
    int lca_level = 0;
};

LocalSet local_set(const Plan& P, int la, int lb)
{
    LocalSet U;
    U.leaves.push_back(la);
    if (lb != la) U.leaves.push_back(lb);
    U.cols.assign(P.n_levels + 1, {});
    U.nodes.assign(P.n_levels + 1, {});
    std::vector<char> seen(P.node_lo.size(), 0);
    for (int l : U.leaves) {
        for (int k = 0; k < P.anc_stride; ++k) {
            const int t = P.leaf_anc[(size_t)l * P.anc_stride + k];
            if (t < 0) break;
            if (seen[t]) {   // shared from here up: the lowest common ancestor
                if (U.lca_level == 0) U.lca_level = P.node_level[t];
                break;
            }
            seen[t] = 1;
            const int h = P.node_level[t];
            bool hit_any = false;
            for (int pp = P.node_pan0[t]; pp < P.node_pan0[t] + P.node_npan[t]; ++pp) {
                bool hit = false;
                for (int x : U.leaves) hit |= P.leaf_lo[x] >= P.pan_lo[pp] && P.leaf_lo[x] < P.pan_lo[pp] + P.pan_n[pp];
                if (!hit) continue;
                hit_any = true;
                for (int q = 0; q < P.pan_m[pp]; ++q) U.cols[h].push_back(P.pan_col0[pp] + q);
            }
            if (hit_any) U.nodes[h].push_back(t);
        }
    }
    return U;
}

// FP64 rebuild of a local set on the device, then the low-precision copies and the stored change
// set (its u vectors depend on the base inverse).  Returns the kernels' flags in *flags.
hinv_status rebuild_local(hinv_ctx& c, const LocalSet& U, hipStream_t s, int* flags)
{
    const Plan& P = c.P;
    std::vector<int> lst(U.leaves);
    std::vector<int> col_at(P.n_levels + 1, 0), node_at(P.n_levels + 1, 0);
    std::vector<std::vector<int>> ord(P.n_levels + 1);
    for (int h = 1; h <= P.n_levels; ++h) {
        col_at[h] = (int)lst.size();
        lst.insert(lst.end(), U.cols[h].begin(), U.cols[h].end());
        node_at[h] = (int)lst.size();
        ord[h] = order_nodes(P, U.nodes[h]);
        lst.insert(lst.end(), ord[h].begin(), ord[h].end());
    }
    HIP_TRY(hipMemcpyAsync(c.upd_list, lst.data(), sizeof(int) * lst.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(c.d_flags, 0, sizeof(int), s));
    launch_leaf_inverse(c.H, c.d_flags, s, c.upd_list, (int)U.leaves.size());
    for (int h = 1; h <= P.n_levels; ++h) {
        const int nc = (int)U.cols[h].size();
        if (nc > 0) launch_build_z(c.H, h, nc, s, c.upd_list + col_at[h]);
        hinv_status st = invert_level(c, h, c.upd_list + node_at[h], ord[h], s);
        if (st != HINV_OK) return st;
    }
    convert_low(c, s);
    HIP_TRY(hipGetLastError());
    for (int j = 0; j < (int)c.mod_a.size(); ++j) {
        hinv_status st = store_mod_u(c, j, s);
        if (st != HINV_OK) return st;
    }
    if (!c.mod_a.empty()) launch_smw_capacitance(c.M, c.d_flags, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(flags, c.d_flags, sizeof(int), hipMemcpyDeviceToHost));
    return HINV_OK;
}

hinv_status plan_and_size(const hinv_csr* G, const hinv_tree* T, const hinv_options* o, int n_sets, int R,
                          int max_nrhs, hinv_ctx& c, size_t* bytes)
{
    hinv_status st = make_plan(G, T, c.P);
    if (st != HINV_OK) return st;
    c.opt = *o;
    Arena A;
    carve_hier(c, A, n_sets, R, max_nrhs);
    *bytes = A.off + kAlign;
    return HINV_OK;
}

// One value change of G between buses a and b (b = -1: a to ground) and the
// entries and old values it touched, so that it can be undone bit for bit.
struct LineEdit {
    int e_aa = -1, e_bb = -1, e_ab = -1, e_ba = -1, ca = -1, cb = -1;
    double aa = 0.0, bb = 0.0, ab = 0.0, w = 0.0;    // values before the change
    LocalSet U;
};

hinv_status set_line_values(hinv_ctx& c, const LineEdit& E, double aa, double bb, double ab, double w, hipStream_t s)
{
    Plan& P = c.P;
    P.cv[E.e_aa] = aa;
    HIP_TRY(hipMemcpyAsync((void*)(c.H.cv + E.e_aa), &P.cv[E.e_aa], sizeof(double), hipMemcpyHostToDevice, s));
    if (E.e_bb >= 0) {
        P.cv[E.e_bb] = bb;
        HIP_TRY(hipMemcpyAsync((void*)(c.H.cv + E.e_bb), &P.cv[E.e_bb], sizeof(double), hipMemcpyHostToDevice, s));
    }
    if (E.e_ab >= 0) {
        P.cv[E.e_ab] = ab; P.cv[E.e_ba] = ab;
        HIP_TRY(hipMemcpyAsync((void*)(c.H.cv + E.e_ab), &P.cv[E.e_ab], sizeof(double), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void*)(c.H.cv + E.e_ba), &P.cv[E.e_ba], sizeof(double), hipMemcpyHostToDevice, s));
    }
    if (E.ca >= 0) {
        P.col_w[E.ca] = w; P.col_w[E.cb] = w;
        HIP_TRY(hipMemcpyAsync((void*)(c.H.col_w + E.ca), &P.col_w[E.ca], sizeof(double), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void*)(c.H.col_w + E.cb), &P.col_w[E.cb], sizeof(double), hipMemcpyHostToDevice, s));
    }
    return HINV_OK;
}

// Restore the values an edit_line changed and rebuild the same local set:
// the inverse is then bitwise the one before the change.
hinv_status undo_line(hinv_ctx& c, const LineEdit& E, hipStream_t s)
{
    hinv_status st = set_line_values(c, E, E.aa, E.bb, E.ab, E.w, s);
    if (st != HINV_OK) return st;
    int back = 0;
    st = rebuild_local(c, E.U, s, &back);
    if (st != HINV_OK) return st;
    HIP_TRY(hipMemsetAsync(c.d_flags, 0, sizeof(int), s));
    HIP_TRY(hipStreamSynchronize(s));
    if (back & (kFlagNotSPD | kFlagSingular)) return fail(HINV_E_DEVICE, "restoring the inverse failed");
    return HINV_OK;
}

// Algorithm 2 made exact: change G by delta_g (e_a - e_b)(e_a - e_b)^T and
// rebuild the two leaves and the paths up to their lowest common ancestor.
// On an indefinite or singular result the old inverse is restored.
hinv_status edit_line(hinv_ctx& c, int32_t a, int32_t b, double delta_g, hipStream_t s, LineEdit& E)
{
    Plan& P = c.P;
    const int n = P.n;
    if (a < 0 || a >= n || b < -1 || b >= n || a == b) return fail(HINV_E_INVALID, "bad buses (%d, %d)", a, b);
    if (!isfinite(delta_g) || delta_g == 0.0) return fail(HINV_E_INVALID, "delta_g must be finite and non-zero");
    const int ra = P.iperm[a], rb = b >= 0 ? P.iperm[b] : -1;
    auto entry = [&](int r, int col) {
        for (int e = P.rp[r]; e < P.rp[r + 1]; ++e)
            if (P.ci[e] == col) return e;
        return -1;
    };
    E.e_aa = entry(ra, ra);
    E.e_bb = rb >= 0 ? entry(rb, rb) : -1;
    E.e_ab = rb >= 0 ? entry(ra, rb) : -1;
    E.e_ba = rb >= 0 ? entry(rb, ra) : -1;
    if (rb >= 0 && (E.e_ab < 0 || E.e_ba < 0))
        return fail(HINV_E_NO_SUCH_LINE, "G has no entry between buses %d and %d; a new coupling needs a rebuild", a, b);
    const int la = P.row_leaf[ra], lb = rb >= 0 ? P.row_leaf[rb] : la;
    // the coupling column pair of a line between two leaves
    E.ca = E.cb = -1;
    if (la != lb) {
        for (int g = 0; g < (int)P.col_row.size() && E.ca < 0; ++g)
            if (P.col_row[g] == ra && P.col_row[P.col_partner[g]] == rb) { E.ca = g; E.cb = P.col_partner[g]; }
        if (E.ca < 0)
            return fail(HINV_E_NO_SUCH_LINE, "buses %d and %d are in different leaves and G has no line between "
                        "them; a new coupling needs a rebuild", a, b);
    }
    E.aa = P.cv[E.e_aa];
    E.bb = E.e_bb >= 0 ? P.cv[E.e_bb] : 0.0;
    E.ab = E.e_ab >= 0 ? P.cv[E.e_ab] : 0.0;
    E.w = E.ca >= 0 ? P.col_w[E.ca] : 0.0;
    double new_ab = E.ab - delta_g;
    if (E.e_ab >= 0) {
        if (fabs(new_ab) <= 1e-12 * fabs(delta_g)) new_ab = 0.0;
        if (new_ab > 0.0)
            return fail(HINV_E_NO_SUCH_LINE, "no line of conductance %g between %d and %d", -delta_g, a, b);
    }
    E.U = local_set(P, la, lb);
    hinv_status st = set_line_values(c, E, E.aa + delta_g, E.bb + delta_g, new_ab, sqrt(fabs(new_ab)), s);
    if (st != HINV_OK) return st;
    int flags = 0;
    st = rebuild_local(c, E.U, s, &flags);
    if (st != HINV_OK) return st;
    if (flags & kFlagBarrier) return fail(HINV_E_DEVICE, "a workgroup team of the rebuild timed out at a barrier");
    if (flags & (kFlagNotSPD | kFlagSingular)) {
        st = undo_line(c, E, s);
        if (st != HINV_OK) return st;
        return fail((flags & kFlagNotSPD) ? HINV_E_NOT_SPD : HINV_E_SINGULAR,
                    "the change makes G (or G with the stored line changes) indefinite or singular");
    }
    return HINV_OK;
}

void fill_update_info(const Plan& P, const LocalSet& U, hinv_update_info* out)
{
    out->lca_level = U.lca_level;
    out->leaves = (int32_t)U.leaves.size();
    out->columns = 0;
    out->nodes = 0;
    for (int hh = 1; hh <= P.n_levels; ++hh) {
        out->columns += (int32_t)U.cols[hh].size();
        out->nodes += (int32_t)U.nodes[hh].size();
    }
}

// ------------------------------------------------------------------------------------------
// Static device scratch of the allocation-free solve (hinv_solve_noalloc).  Each GPU the library
// runs on holds one copy of this array for the life of the process.  In host code its name is only a
// stand-in for the symbol: the device address of each GPU's copy comes from hipGetSymbolAddress, once
// per device, and only that address is handed to kernels.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// The current device's copy of the scratch array (looked up on the first call per device).
hinv_status scratch_of_current_device(void** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(HINV_E_DEVICE, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(HINV_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HINV_OK;
}

// Scratch bytes of one allocation-free solve: permuted input and output, the level values, and with
// refinement the residual, the correction and the per-column stats.
size_t noalloc_bytes(const hinv_ctx& c, int nrhs)
{
    const size_t n = (size_t)c.P.n, nc = c.P.col_row.size(), k = (size_t)nrhs;
    auto al = [](size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); };
    size_t b = 2 * al(sizeof(double) * n * k) + al(sizeof(double) * (nc > 0 ? nc : 1) * k);
    b += 2 * al(sizeof(double) * n * k) + al(sizeof(unsigned long long) * k);
    return b;
}

__global__ void k_zero_u64(unsigned long long* p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

}  // namespace

// =============================== C ABI =====================================
extern "C" {

const char* hinv_last_error(void) { return g_err.c_str(); }

hinv_status hinv_workspace_size(const hinv_csr* G, const hinv_tree* tree, const hinv_options* opt, size_t* bytes)
{
    if (!bytes) return fail(HINV_E_INVALID, "bytes is NULL");
    hinv_status st = check_options(opt, 1);
    if (st != HINV_OK) return st;
    std::unique_ptr<hinv_ctx> c(new (std::nothrow) hinv_ctx);
    if (!c) return fail(HINV_E_NO_MEMORY, "host allocation failed");
    return plan_and_size(G, tree, opt, 1, std::max(1, opt->max_mod_rank), opt->max_nrhs, *c, bytes);
}

hinv_status hinv_build(const hinv_csr* G, const hinv_tree* tree, const hinv_options* opt, void* d_ws,
                       size_t ws_bytes, void* stream, hinv_handle* out)
{
    if (!out) return fail(HINV_E_INVALID, "out is NULL");
    *out = nullptr;
    hinv_status st = check_options(opt, 1);
    if (st != HINV_OK) return st;
    std::unique_ptr<hinv_ctx> c(new (std::nothrow) hinv_ctx);
    if (!c) return fail(HINV_E_NO_MEMORY, "host allocation failed");
    size_t need = 0;
    const int R = std::max(1, opt->max_mod_rank);
    st = plan_and_size(G, tree, opt, 1, R, opt->max_nrhs, *c, &need);
    if (st != HINV_OK) return st;
    if (!d_ws) return fail(HINV_E_INVALID, "workspace is NULL");
    if (ws_bytes < need) return fail(HINV_E_NO_MEMORY, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    Arena A;
    A.base = (char*)d_ws;
    carve_hier(*c, A, 1, R, opt->max_nrhs);
    c->M.R = opt->max_mod_rank;     // 0 disables the correction entirely
    st = build_device(*c, (hipStream_t)stream);
    if (st != HINV_OK) return st;
    {   // set-up of the allocation-free solve's scratch on this device; a failure is reported by that call
        void* ptr = nullptr;
        const std::string keep = g_err;
        if (scratch_of_current_device(&ptr) != HINV_OK) g_err = keep;
    }
    *out = c.release();
    return HINV_OK;
}

hinv_status hinv_modify_line(hinv_handle h, int32_t a, int32_t b, double delta_g, void* stream)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    hinv_ctx& c = *h;
    hipStream_t s = (hipStream_t)stream;
    const int n = c.P.n;
    if (a < 0 || a >= n || b < -1 || b >= n || a == b) return fail(HINV_E_INVALID, "bad buses (%d, %d)", a, b);
    if (!isfinite(delta_g) || delta_g == 0.0) return fail(HINV_E_INVALID, "delta_g must be finite and non-zero");
    const int cnt = (int)c.mod_a.size();
    if (cnt >= c.opt.max_mod_rank) return fail(HINV_E_RANK_LIMIT, "already %d changes (max_mod_rank)", cnt);
    const int ra = c.P.iperm[a], rb = b >= 0 ? c.P.iperm[b] : -1;
    if (delta_g < 0 && rb >= 0) {   // removing conductance needs that much conductance between a and b
        double gab = 0.0;
        for (int e = c.P.rp[ra]; e < c.P.rp[ra + 1]; ++e)
            if (c.P.ci[e] == rb) gab = -c.P.cv[e];
        for (int j = 0; j < cnt; ++j)
            if ((c.mod_a[j] == ra && c.mod_b[j] == rb) || (c.mod_a[j] == rb && c.mod_b[j] == ra)) gab += c.mod_dg[j];
        if (gab + delta_g < -1e-12 * fabs(delta_g))
            return fail(HINV_E_NO_SUCH_LINE, "no line of conductance %g between %d and %d", -delta_g, a, b);
    }
    // u = G0^{-1} w, w = e_a - e_b, by one FP64 apply
    c.mod_a.push_back(ra); c.mod_b.push_back(rb); c.mod_dg.push_back(delta_g); c.mod_act.push_back(INT32_MIN);
    {
        hinv_status st = store_mod_u(c, cnt, s);
        if (st != HINV_OK) {
            c.mod_a.pop_back(); c.mod_b.pop_back(); c.mod_dg.pop_back(); c.mod_act.pop_back();
            return st;
        }
    }
    std::vector<int> cntv{cnt + 1};
    HIP_TRY(hipMemcpyAsync(c.m_a, c.mod_a.data(), sizeof(int) * (cnt + 1), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c.m_b, c.mod_b.data(), sizeof(int) * (cnt + 1), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c.m_dg, c.mod_dg.data(), sizeof(double) * (cnt + 1), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c.m_act, c.mod_act.data(), sizeof(int) * (cnt + 1), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c.m_count, cntv.data(), sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(c.d_flags, 0, sizeof(int), s));
    launch_smw_capacitance(c.M, c.d_flags, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    int flags = 0;
    HIP_TRY(hipMemcpy(&flags, c.d_flags, sizeof(int), hipMemcpyDeviceToHost));
    if (flags & (kFlagNotSPD | kFlagSingular)) {
        // roll back
        c.mod_a.pop_back(); c.mod_b.pop_back(); c.mod_dg.pop_back(); c.mod_act.pop_back();
        std::vector<int> back{cnt};
        HIP_TRY(hipMemcpy(c.m_count, back.data(), sizeof(int), hipMemcpyHostToDevice));
        return fail(HINV_E_NOT_SPD, "the change makes G indefinite or singular");
    }
    return HINV_OK;
}

hinv_status hinv_update_line(hinv_handle h, int32_t a, int32_t b, double delta_g, void* stream,
                             hinv_update_info* out)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    LineEdit ed;
    hinv_status st = edit_line(*h, a, b, delta_g, (hipStream_t)stream, ed);
    if (st != HINV_OK) return st;
    if (out) fill_update_info(h->P, ed.U, out);
    return HINV_OK;
}

hinv_status hinv_solve(hinv_handle h, const double* d_i, double* d_v, int32_t nrhs, int32_t ld, void* stream)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    hinv_ctx& c = *h;
    if (nrhs < 0 || nrhs > c.opt.max_nrhs) return fail(HINV_E_INVALID, "nrhs %d outside 0..%d", nrhs, c.opt.max_nrhs);
    if (ld < c.P.n) return fail(HINV_E_INVALID, "ld %d < n %d", ld, c.P.n);
    if (nrhs == 0) return HINV_OK;
    if (!d_i || !d_v) return fail(HINV_E_INVALID, "NULL vector");
    hipStream_t s = (hipStream_t)stream;
    launch_permute_in(c.P.n, nrhs, c.d_perm, d_i, ld, c.X, s);
    solve_new_order(c, c.X, c.Xo, nrhs, 0, nullptr, s);
    launch_permute_out(c.P.n, nrhs, c.d_perm, c.Xo, d_v, ld, s);
    HIP_TRY(hipGetLastError());
    return HINV_OK;
}

hinv_status hinv_solve_noalloc(hinv_handle h, const double* d_i, double* d_v, int32_t nrhs, int32_t ld, void* stream)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    hinv_ctx& c = *h;
    if (nrhs < 0) return fail(HINV_E_INVALID, "nrhs %d < 0", nrhs);
    if (ld < c.P.n) return fail(HINV_E_INVALID, "ld %d < n %d", ld, c.P.n);
    if (nrhs == 0) return HINV_OK;
    if (!d_i || !d_v) return fail(HINV_E_INVALID, "NULL vector");
    const size_t need = noalloc_bytes(c, nrhs);
    if (need > kNoAllocScratchBytes)
        return fail(HINV_E_INVALID, "%d right-hand sides of order %d need %zu bytes of scratch; the static scratch "
                    "holds %zu", nrhs, c.P.n, need, kNoAllocScratchBytes);
    void* base = nullptr;
    hinv_status st = scratch_of_current_device(&base);
    if (st != HINV_OK) return st;
    Arena A;
    A.base = (char*)base;
    const int64_t nk = (int64_t)c.P.n * nrhs;
    double* X = A.take<double>(nk);
    double* Xo = A.take<double>(nk);
    SolveTemps w{};
    w.Y = A.take<double>((int64_t)std::max<size_t>(c.P.col_row.size(), 1) * nrhs);
    w.Rv = A.take<double>(nk);
    w.D = A.take<double>(nk);
    w.stats = A.take<unsigned long long>(nrhs);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero_u64, dim3((nrhs + 255) / 256), dim3(256), 0, s, w.stats, nrhs);
    launch_permute_in(c.P.n, nrhs, c.d_perm, d_i, ld, X, s);
    solve_new_order(c, w, X, Xo, nrhs, 0, nullptr, s);
    launch_permute_out(c.P.n, nrhs, c.d_perm, Xo, d_v, ld, s);
    HIP_TRY(hipGetLastError());
    return HINV_OK;
}

// Workspace of hinv_solve_gmres (base == nullptr: measure only).
struct GmresWs {
    double *B, *X, *R, *D, *W, *Zero, *V, *Z, *Y, *dots, *nrm, *Hs, *cs, *sn, *g, *res, *y;
    unsigned long long* stats;
};

static void carve_gmres(const hinv_ctx& c, Arena& A, int nrhs, int m, GmresWs& w)
{
    const int64_t nk = (int64_t)c.P.n * nrhs;
    w.B = A.take<double>(nk); w.X = A.take<double>(nk); w.R = A.take<double>(nk); w.D = A.take<double>(nk);
    w.W = A.take<double>(nk); w.Zero = A.take<double>(nk);
    w.V = A.take<double>((int64_t)(m + 1) * nk);
    w.Z = A.take<double>((int64_t)m * nk);
    w.Y = A.take<double>((int64_t)std::max<size_t>(c.P.col_row.size(), 1) * nrhs);
    w.dots = A.take<double>((int64_t)2 * (m + 1) * nrhs);
    w.nrm = A.take<double>(nrhs);
    w.Hs = A.take<double>((int64_t)(m + 1) * m * nrhs);
    w.cs = A.take<double>((int64_t)m * nrhs); w.sn = A.take<double>((int64_t)m * nrhs);
    w.g = A.take<double>((int64_t)(m + 1) * nrhs);
    w.res = A.take<double>(nrhs);
    w.y = A.take<double>((int64_t)m * nrhs);
    w.stats = A.take<unsigned long long>(nrhs);
}

hinv_status hinv_gmres_workspace_size(hinv_handle h, int32_t nrhs, int32_t m, size_t* bytes)
{
    if (!h || !bytes) return fail(HINV_E_INVALID, "NULL argument");
    if (nrhs < 1 || m < 1 || m > kGmresMaxInner)
        return fail(HINV_E_INVALID, "nrhs %d < 1 or m %d outside 1..%d", nrhs, m, kGmresMaxInner);
    Arena A;
    GmresWs w{};
    carve_gmres(*h, A, nrhs, m, w);
    *bytes = A.off + kAlign;
    return HINV_OK;
}

hinv_status hinv_solve_gmres(hinv_handle h, const double* d_i, double* d_v, int32_t nrhs, int32_t ld, int32_t m,
                             int32_t max_outer, int32_t smooth, double inner_tol, double rel_tol, void* d_ws,
                             size_t ws_bytes, void* stream, hinv_gmres_info* info)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    hinv_ctx& c = *h;
    if (info) *info = hinv_gmres_info{0, 0, 0.0};
    if (nrhs < 1 || m < 1 || m > kGmresMaxInner || max_outer < 0 || smooth < 0 || smooth > 16)
        return fail(HINV_E_INVALID, "nrhs %d < 1, m %d outside 1..%d, max_outer %d < 0 or smooth %d outside 0..16",
                    nrhs, m, kGmresMaxInner, max_outer, smooth);
    if (ld < c.P.n) return fail(HINV_E_INVALID, "ld %d < n %d", ld, c.P.n);
    if (!d_i || !d_v || !d_ws) return fail(HINV_E_INVALID, "NULL vector or workspace");
    if (!(inner_tol > 0.0 && inner_tol < 1.0) || !(rel_tol > 0.0))
        return fail(HINV_E_INVALID, "inner_tol must be in (0, 1) and rel_tol positive");
    size_t need = 0;
    hinv_status st = hinv_gmres_workspace_size(h, nrhs, m, &need);
    if (st != HINV_OK) return st;
    if (ws_bytes < need) return fail(HINV_E_NO_MEMORY, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    Arena A;
    A.base = (char*)d_ws;
    GmresWs w{};
    carve_gmres(c, A, nrhs, m, w);
    const int n = c.P.n;
    const int64_t nk = (int64_t)n * nrhs;
    const int prec = c.opt.prec;
    hipStream_t s = (hipStream_t)stream;
    const SolveTemps tmp{w.Y, w.R, w.D, w.stats};
    // M v: the stored inverse in its storage precision, then `smooth` damped-Jacobi sweeps (W as scratch)
    auto apply_m = [&](const double* Vin, double* Zout) {
        precond(c, tmp, prec, Vin, Zout, nrhs, 0, nullptr, s);
        for (int q = 0; q < smooth; ++q) {
            launch_residual(c.H, c.M, Vin, Zout, w.W, nrhs, 0, nullptr, s);
            launch_gm_jacobi(c.H, nrhs, w.W, 2.0 / 3.0, Zout, s);
        }
    };
    HIP_TRY(hipMemsetAsync(w.Zero, 0, sizeof(double) * nk, s));
    launch_permute_in(n, nrhs, c.d_perm, d_i, ld, w.B, s);
    apply_m(w.B, w.X);                                                  // x_0 = M b
    std::vector<double> beta(nrhs), res(nrhs);
    std::vector<unsigned long long> upd(nrhs);
    int outer = 0, inner_total = 0;
    double last = INFINITY;
    while (outer < max_outer && !(last <= rel_tol)) {
        launch_residual(c.H, c.M, w.B, w.X, w.R, nrhs, 0, nullptr, s);   // r = b - G x, FP64
        launch_gm_norms(n, nrhs, w.R, w.nrm, s);
        launch_gm_start(nrhs, m, w.nrm, w.g, w.res, s);
        launch_gm_scale(n, nrhs, w.R, w.nrm, 1, 1.0, w.V, s);             // v_0 = r / ||r||
        HIP_TRY(hipMemcpyAsync(beta.data(), w.nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        bool zero = true;
        for (double b : beta) zero = zero && b == 0.0;
        if (zero) { last = 0.0; break; }
        int j = 0;
        while (j < m) {
            double* Vj = w.V + (int64_t)j * nk;
            double* Zj = w.Z + (int64_t)j * nk;
            apply_m(Vj, Zj);                                                  // z_j = M v_j
            launch_residual(c.H, c.M, w.Zero, Zj, w.W, nrhs, 0, nullptr, s);   // W = -G z_j = -w
            for (int pass = 0; pass < 2; ++pass) {                            // w -= sum h v_i, twice
                double* h2 = w.dots + pass * (m + 1);
                launch_gm_dots(n, nrhs, j + 1, w.V, w.W, -1.0, h2, 2 * (m + 1), s);
                launch_gm_update(n, nrhs, j + 1, w.V, h2, 2 * (m + 1), 1.0, w.W, s);
            }
            launch_gm_norms(n, nrhs, w.W, w.nrm, s);
            launch_gm_givens(nrhs, m, j, w.dots, w.nrm, w.Hs, w.cs, w.sn, w.g, w.res, s);
            launch_gm_scale(n, nrhs, w.W, w.nrm, 1, -1.0, w.V + (int64_t)(j + 1) * nk, s);   // v_{j+1} = w/||w||
            ++j;
            ++inner_total;
            HIP_TRY(hipMemcpyAsync(res.data(), w.res, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            bool done = true;
            for (int k = 0; k < nrhs; ++k) done = done && !(res[k] > inner_tol * beta[k]);
            if (done) break;
        }
        launch_gm_backsolve(nrhs, m, j, w.Hs, w.g, w.y, s);
        HIP_TRY(hipMemsetAsync(w.D, 0, sizeof(double) * nk, s));
        launch_gm_update(n, nrhs, j, w.Z, w.y, m, 1.0, w.D, s);             // d = sum_j y_j z_j
        hipLaunchKernelGGL(k_zero_u64, dim3((nrhs + 255) / 256), dim3(256), 0, s, w.stats, nrhs);
        launch_axpy_stats(n, nrhs, w.X, w.D, w.stats, 1e300, c.d_flags, s);  // x += d, ||d||/||x|| per column
        HIP_TRY(hipMemcpyAsync(upd.data(), w.stats, sizeof(unsigned long long) * nrhs, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        last = 0.0;
        for (unsigned long long u : upd) {
            double r;
            memcpy(&r, &u, sizeof r);
            last = std::max(last, r);
        }
        ++outer;
    }
    launch_permute_out(n, nrhs, c.d_perm, w.X, d_v, ld, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    c.applies += (int64_t)nrhs * (1 + inner_total) * (1 + smooth);
    if (info) *info = hinv_gmres_info{outer, inner_total, last};
    if (!(last <= rel_tol))
        return fail(HINV_E_NO_CONVERGENCE, "GMRES refinement: last update %g above rel_tol %g after %d corrections",
                    last, rel_tol, outer);
    return HINV_OK;
}

hinv_status hinv_sync_status(hinv_handle h)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    int flags[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpy(flags, h->d_flags, sizeof flags, hipMemcpyDeviceToHost));
    int zero[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpy(h->d_flags, zero, sizeof zero, hipMemcpyHostToDevice));
    if (flags[0] & kFlagNoConv) return fail(HINV_E_NO_CONVERGENCE, "refinement did not converge");
    if (flags[0] & (kFlagNotSPD | kFlagNaN)) return fail(HINV_E_NOT_SPD, "non-finite or indefinite result");
    return HINV_OK;
}

hinv_status hinv_get_info(hinv_handle h, hinv_info_t* out)
{
    if (!h || !out) return fail(HINV_E_INVALID, "NULL argument");
    const Plan& P = h->P;
    out->n = P.n;
    out->n_leaves = (int64_t)P.leaf_lo.size();
    out->n_internal = (int64_t)P.node_lo.size();
    out->n_levels = P.n_levels;
    out->n_cols = (int64_t)P.col_row.size();
    int64_t le = 0, ze = 0, se = 0;
    for (int x : P.leaf_n) le += (int64_t)x * x;
    for (size_t i = 0; i < P.pan_n.size(); ++i) ze += (int64_t)P.pan_n[i] * P.pan_m[i];
    for (int m : P.node_m) se += (int64_t)m * m;
    out->leaf_entries = le;
    out->z_entries = ze;
    out->s_entries = se;
    out->max_leaf = P.max_leaf;
    out->max_cols = P.max_cols;
    // FLOP counts of the apply and the build, from the plan
    std::vector<double> node_upd(P.node_lo.size(), 0.0);   // one Woodbury update of a vector at node t
    double ap = 0.0, bu = 0.0;
    for (int x : P.leaf_n) { ap += 2.0 * x * x; bu += 2.0 * (double)x * x * x; }
    for (size_t t = 0; t < P.node_lo.size(); ++t) {
        const double m = P.node_m[t];
        double u = m + 2.0 * m * m;
        for (int pp = P.node_pan0[t]; pp < P.node_pan0[t] + P.node_npan[t]; ++pp) u += 2.0 * P.pan_n[pp] * P.pan_m[pp];
        node_upd[t] = u;
        ap += u;
        bu += m * m + 2.0 * m * m * m;
    }
    for (size_t g = 0; g < P.col_row.size(); ++g) {
        const int l = P.row_leaf[P.col_row[g]];
        const int h = P.node_level[P.col_node[g]];
        bu += P.leaf_n[l];
        for (int k = 0; k < P.anc_stride; ++k) {
            const int t = P.leaf_anc[(size_t)l * P.anc_stride + k];
            if (t < 0 || P.node_level[t] >= h) break;
            bu += node_upd[t];
        }
    }
    out->apply_flops = ap;
    out->build_flops = bu;
    return HINV_OK;
}

hinv_status hinv_destroy(hinv_handle h)
{
    delete h;
    return HINV_OK;
}

}  // extern "C"

// =========================== EMT time stepping ==============================
struct emt_ctx {
    hinv_ctx hc;                 // hierarchy of G; change set k belongs to case k
    EmtDev E{};
    RecParams* d_rec = nullptr;
    int n = 0, nbr = 0, n_cases = 0, R = 0;
    std::vector<int> fr_p, to_p;
    std::vector<double> g;
    std::vector<std::vector<std::pair<int, int>>> losses;   // per case: (step, branch), sorted
    int64_t step = 1;
    unsigned long long* d_applies = nullptr;   // [n_cases] fused-path apply counters
    int64_t* d_clock = nullptr;
    int64_t clock_cap = 0;
    double* gscr = nullptr;      // [4 * n * n_cases] case vectors when they do not fit LDS (serving)
    // new-order network data kept for the team plan
    std::vector<int> inc_ptr, inc_br, src_ptr;
    std::vector<double> alpha, samp, sph, gC;
    int engine = 1;              // 1 per-kernel, 2 one workgroup per case, 3 team, 4 panel, 5 level
    // team engine
    bool team_ok = false;
    int team_nx_cap = 0;
    std::vector<int> tw_nxu, txupd, tuzo;   // team: X rows whose final values a workgroup uses
    std::vector<int> ttcso, ttcld, tylist, tw_ny;   // team: columns whose y a workgroup computes, S^{-1} rows
    std::vector<int> tw_lo, tw_nl, tw_nx, tw_nb, txrow, txzo, txpm, txpc, tozo, topm, topc, topan, txpan, txpos, torp,
        tocol, tbglob, tbf, tbt, tbown, tiptr, tibr, tsptr;
    std::vector<double> toval, tbg, tbal, tsamp, tsph;
    std::vector<int> tosrc;      // CSR entry (plus one, 0 = padding) of each toval value
    std::vector<int> tcsop;
    std::vector<int> taoff, talo, talen, tcpan;   // rows a_g of the two-phase coupling levels
    TeamDev TD{};
    // panel engine (cases in panels of kPanelCases, one workgroup per leaf per panel)
    bool panel_ok = false;
    std::vector<int> phbft, phlost, pxzsrc, pw_xz;
    std::vector<int> pw_nx, pw_ny, pw_nt, pw_np, pxrow, pxcol, pxzo, pxpm, pxps, pxpan, plpa, plpb, pcpan, ppubr, ppubg,
        pyslot, ptk0, ptnk, ptfo, pttile, pttp, pttl, pwtask;
    PanelDev PD{};
    // level engine (one case, distributed coupling levels)
    bool level_ok = false;
    int level_nx_cap = 0;
    std::vector<int> lw_nx, loptr, locl, lorow, losoff, lxrow, llpa, llpb;
    LevelDev LD{};
    // three-phase networks (emt3_create): rows are bus phases (row 3a + p of the caller's order), branch
    // 3l + p is phase p of line l; per line the 3x3 companion admittance Y, history weight A = I - 2 R Y
    // and impedance Z = Y^{-1} (row-major)
    int ph = 1;
    int n_lines = 0;
    std::vector<double> y3, a3, z3;
    double* m_d3 = nullptr;
    double* m_dinv3 = nullptr;
    // checkpoints: fingerprint of the caller's network and the base-matrix changes made since creation
    uint64_t net_hash = 0;
    std::string table_error;     // first failed bounds check of an engine's tables (empty: all in bounds)
    struct BaseChange {
        int32_t a, b;
        double dg;
    };
    std::vector<BaseChange> base_log;
};

// Three-phase network parameters of emt3_create.
struct Phase3 {
    double mu;           // mutual / self inductance of every line
    double shift[3];     // source phase shift of each phase
};

namespace {

hinv_status check_network(const emt_network* N)
{
    if (!N) return fail(HINV_E_INVALID, "network is NULL");
    if (N->n_bus < 1 || N->n_branch < 0 || N->n_src < 0) return fail(HINV_E_INVALID, "negative or zero sizes");
    if (!(N->dt > 0.0) || !isfinite(N->dt)) return fail(HINV_E_INVALID, "dt must be positive");
    if (!isfinite(N->freq)) return fail(HINV_E_INVALID, "freq must be finite");
    if (N->n_branch > 0 && (!N->from || !N->to || !N->R || !N->L))
        return fail(HINV_E_INVALID, "branch arrays must not be NULL");
    if (!N->C) return fail(HINV_E_INVALID, "C must not be NULL");
    if (N->n_src > 0 && (!N->src_bus || !N->amp || !N->phase)) return fail(HINV_E_INVALID, "source arrays must not be NULL");
    for (int e = 0; e < N->n_branch; ++e) {
        const int a = N->from[e], b = N->to[e];
        if (a < 0 || a >= N->n_bus || b < 0 || b >= N->n_bus || a == b)
            return fail(HINV_E_INVALID, "branch %d has bad buses (%d, %d)", e, a, b);
        const double z = N->R[e] + 2.0 * N->L[e] / N->dt;
        if (!(N->R[e] >= 0.0) || !(N->L[e] >= 0.0) || !(z > 0.0) || !isfinite(z))
            return fail(HINV_E_INVALID, "branch %d has bad R/L", e);
    }
    for (int a = 0; a < N->n_bus; ++a)
        if (!(N->C[a] >= 0.0) || !isfinite(N->C[a])) return fail(HINV_E_INVALID, "C[%d] is negative or not finite", a);
    for (int q = 0; q < N->n_src; ++q)
        if (N->src_bus[q] < 0 || N->src_bus[q] >= N->n_bus || !isfinite(N->amp[q]) || !isfinite(N->phase[q]))
            return fail(HINV_E_INVALID, "source %d is invalid", q);
    return HINV_OK;
}

hinv_status check_cases(const emt_cases* C, int nbr, int R, std::vector<std::vector<std::pair<int, int>>>& out)
{
    if (!C || C->n_cases < 1) return fail(HINV_E_INVALID, "need at least one case");
    out.assign(C->n_cases, {});
    if (!C->loss_ptr) return HINV_OK;
    if (C->loss_ptr[0] != 0) return fail(HINV_E_INVALID, "loss_ptr[0] != 0");
    for (int k = 0; k < C->n_cases; ++k) {
        const int b = C->loss_ptr[k], e = C->loss_ptr[k + 1];
        if (e < b) return fail(HINV_E_INVALID, "loss_ptr not non-decreasing at case %d", k);
        if (e > b && (!C->loss_step || !C->loss_branch)) return fail(HINV_E_INVALID, "loss arrays are NULL");
        if (e - b > R) return fail(HINV_E_RANK_LIMIT, "case %d has %d losses (max_mod_rank %d)", k, e - b, R);
        for (int j = b; j < e; ++j) {
            const int br = C->loss_branch[j], st = C->loss_step[j];
            if (br < 0 || br >= nbr) return fail(HINV_E_INVALID, "case %d loses unknown branch %d", k, br);
            if (st < 1) return fail(HINV_E_INVALID, "case %d: loss step %d < 1", k, st);
            for (auto& x : out[k])
                if (x.second == br) return fail(HINV_E_INVALID, "case %d loses branch %d twice", k, br);
            out[k].push_back({st, br});
        }
        std::stable_sort(out[k].begin(), out[k].end());
    }
    return HINV_OK;
}

// Nodal conductance matrix of the network (trapezoidal companions), CSR with sorted columns.
void assemble_csr(const emt_network* N, std::vector<int>& rp, std::vector<int>& ci, std::vector<double>& cv)
{
    const int n = N->n_bus;
    struct T { int r, c; double v; };
    std::vector<T> t;
    t.reserve((size_t)n + 4 * (size_t)N->n_branch);
    for (int a = 0; a < n; ++a) t.push_back({a, a, 2.0 * N->C[a] / N->dt});
    for (int e = 0; e < N->n_branch; ++e) {
        const double g = 1.0 / (N->R[e] + 2.0 * N->L[e] / N->dt);
        const int a = N->from[e], b = N->to[e];
        t.push_back({a, a, g});
        t.push_back({b, b, g});
        t.push_back({a, b, -g});
        t.push_back({b, a, -g});
    }
    std::stable_sort(t.begin(), t.end(), [](const T& x, const T& y) { return x.r != y.r ? x.r < y.r : x.c < y.c; });
    rp.assign(n + 1, 0);
    ci.clear();
    cv.clear();
    int last_row = -1;
    for (size_t i = 0; i < t.size(); ++i) {
        if (t[i].r == last_row && ci.back() == t[i].c) {
            cv.back() += t[i].v;          // parallel branches and the diagonal sum up
        } else {
            ci.push_back(t[i].c);
            cv.push_back(t[i].v);
        }
        last_row = t[i].r;
        rp[t[i].r + 1] = (int)ci.size();
    }
    for (int r = 0; r < n; ++r)
        if (rp[r + 1] < rp[r]) rp[r + 1] = rp[r];
}

// Three-phase G: rows 3a + p; branch e couples the phases of its R-L through mutual inductance
// mutual * L[e], so its companion is the 3x3 admittance Y = (R I + (2/dt) L [(1 - mu) I + mu J])^{-1},
// J the all-ones matrix: with alpha = R + (2L/dt)(1 - mu) and beta = (2L/dt) mu,
// Y = I / alpha - J beta / (alpha (alpha + 3 beta)).  Shunts 2C/dt on each phase.
void assemble_csr3(const emt_network* N, double mu, std::vector<int>& rp, std::vector<int>& ci,
                   std::vector<double>& cv)
{
    const int n = 3 * N->n_bus;
    struct T { int r, c; double v; };
    std::vector<T> t;
    t.reserve((size_t)n + 36 * (size_t)N->n_branch);
    for (int a = 0; a < N->n_bus; ++a)
        for (int p = 0; p < 3; ++p) t.push_back({3 * a + p, 3 * a + p, 2.0 * N->C[a] / N->dt});
    for (int e = 0; e < N->n_branch; ++e) {
        const double zl = 2.0 * N->L[e] / N->dt;
        const double alpha = N->R[e] + zl * (1.0 - mu), beta = zl * mu;
        const double off = -beta / (alpha * (alpha + 3.0 * beta));
        const double dia = 1.0 / alpha + off;
        const int a = N->from[e], b = N->to[e];
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) {
                const double y = (p == q) ? dia : off;
                t.push_back({3 * a + p, 3 * a + q, y});
                t.push_back({3 * b + p, 3 * b + q, y});
                t.push_back({3 * a + p, 3 * b + q, -y});
                t.push_back({3 * b + p, 3 * a + q, -y});
            }
    }
    std::stable_sort(t.begin(), t.end(), [](const T& x, const T& y) { return x.r != y.r ? x.r < y.r : x.c < y.c; });
    rp.assign(n + 1, 0);
    ci.clear();
    cv.clear();
    int last_row = -1;
    for (size_t i = 0; i < t.size(); ++i) {
        if (t[i].r == last_row && ci.back() == t[i].c) {
            cv.back() += t[i].v;
        } else {
            ci.push_back(t[i].c);
            cv.push_back(t[i].v);
        }
        last_row = t[i].r;
        rp[t[i].r + 1] = (int)ci.size();
    }
    for (int r = 0; r < n; ++r)
        if (rp[r + 1] < rp[r]) rp[r + 1] = rp[r];
}

// Device storage of the EMT state (base == nullptr: measure only).
void carve_emt(emt_ctx& c, Arena& A, int n_src)
{
    EmtDev& E = c.E;
    const int n = c.n, nbr = c.nbr, K = c.n_cases, R = c.R;
    E.n = n; E.nbr = nbr; E.n_cases = K; E.R = R;
    E.fr = A.take<int>(nbr); E.to = A.take<int>(nbr);
    E.g = A.take<double>(nbr); E.alpha = A.take<double>(nbr); E.gC = A.take<double>(n);
    E.inc_ptr = A.take<int>(n + 1); E.inc_br = A.take<int>(2 * (int64_t)nbr);
    E.src_ptr = A.take<int>(n + 1); E.src_amp = A.take<double>(n_src); E.src_ph = A.take<double>(n_src);
    E.loss_cnt = A.take<int>(K); E.loss_step = A.take<int>((int64_t)K * R); E.loss_br = A.take<int>((int64_t)K * R);
    E.h = A.take<double>(2 * (int64_t)K * nbr);
    E.hC = A.take<double>((int64_t)K * n); E.b = A.take<double>((int64_t)K * n); E.v = A.take<double>((int64_t)K * n);
    E.step = A.take<int64_t>(1);
    E.done = A.take<unsigned int>(1);
    c.d_rec = A.take<RecParams>(1);
    c.d_applies = A.take<unsigned long long>(K);
    c.gscr = A.take<double>(4 * (int64_t)n * K);
    E.Y3 = E.A3 = nullptr;
    if (c.ph == 3) {
        E.Y3 = A.take<double>(9 * (int64_t)c.n_lines);
        E.A3 = A.take<double>(9 * (int64_t)c.n_lines);
        c.m_d3 = A.take<double>((int64_t)K * R * 3);
        c.m_dinv3 = A.take<double>((int64_t)K * R * 3);
        c.hc.M.grp3 = 1;
        c.hc.M.d3 = c.m_d3;
        c.hc.M.dinv3 = c.m_dinv3;
    }
}

// Network data in the new bus order (kept on the host for uploads and the team plan).
void prepare_network(emt_ctx& c, const emt_network* net)
{
    const Plan& P = c.hc.P;
    const int n = c.n, nbr = c.nbr;
    c.fr_p.assign(nbr, 0); c.to_p.assign(nbr, 0); c.g.assign(nbr, 0.0); c.alpha.assign(nbr, 0.0);
    c.gC.assign(n, 0.0);
    c.inc_ptr.assign(n + 1, 0);
    c.inc_br.assign(2 * (size_t)nbr, 0);
    for (int e = 0; e < nbr; ++e) {
        c.fr_p[e] = P.iperm[net->from[e]];
        c.to_p[e] = P.iperm[net->to[e]];
        const double z2 = 2.0 * net->L[e] / net->dt;
        c.g[e] = 1.0 / (net->R[e] + z2);
        c.alpha[e] = c.g[e] * (z2 - net->R[e]);
        c.inc_ptr[c.fr_p[e] + 1]++;
        c.inc_ptr[c.to_p[e] + 1]++;
    }
    for (int r = 0; r < n; ++r) {
        c.inc_ptr[r + 1] += c.inc_ptr[r];
        c.gC[r] = 2.0 * net->C[P.perm[r]] / net->dt;
    }
    std::vector<int> fill(c.inc_ptr.begin(), c.inc_ptr.end() - 1);
    for (int e = 0; e < nbr; ++e) {
        c.inc_br[fill[c.fr_p[e]]++] = e;
        c.inc_br[fill[c.to_p[e]]++] = e;
    }
    c.src_ptr.assign(n + 1, 0);
    c.samp.assign(net->n_src, 0.0);
    c.sph.assign(net->n_src, 0.0);
    for (int q = 0; q < net->n_src; ++q) c.src_ptr[P.iperm[net->src_bus[q]] + 1]++;
    for (int r = 0; r < n; ++r) c.src_ptr[r + 1] += c.src_ptr[r];
    std::vector<int> sf(c.src_ptr.begin(), c.src_ptr.end() - 1);
    for (int q = 0; q < net->n_src; ++q) {
        const int r = P.iperm[net->src_bus[q]];
        c.samp[sf[r]] = net->amp[q];
        c.sph[sf[r]] = net->phase[q];
        sf[r]++;
    }
}

// Three-phase network data in the new row order.  Line l is a transposed R-L: per phase R, self
// inductance L and mutual inductance mu L between any two phases, so its trapezoidal impedance is
// Z = al I + be J (al = R + (2L/dt)(1 - mu), be = (2L/dt) mu, J all ones) and its companion admittance
// Y = Z^{-1} = I / al - J be / (al (al + 3 be)), the values assemble_csr3 puts into G.  The history
// weight Y ((2/dt) L_e - R I) equals Y (Z - 2 R I) = I - 2 R Y.  Source q drives phase p of its bus with
// its phase plus shift[p].
void prepare_network3(emt_ctx& c, const emt_network* net, const Phase3& p3)
{
    const Plan& P = c.hc.P;
    const int n = c.n, nl = c.n_lines, nbr = c.nbr;
    c.fr_p.assign(nbr, 0); c.to_p.assign(nbr, 0); c.g.assign(nbr, 0.0); c.alpha.assign(nbr, 0.0);
    c.y3.assign(9 * (size_t)nl, 0.0); c.a3.assign(9 * (size_t)nl, 0.0); c.z3.assign(9 * (size_t)nl, 0.0);
    c.gC.assign(n, 0.0);
    c.inc_ptr.assign(n + 1, 0);
    c.inc_br.assign(2 * (size_t)nbr, 0);
    for (int l = 0; l < nl; ++l) {
        const double R = net->R[l], zl = 2.0 * net->L[l] / net->dt;
        const double al = R + zl * (1.0 - p3.mu), be = zl * p3.mu;
        const double off = -be / (al * (al + 3.0 * be));
        const double dia = 1.0 / al + off;
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) {
                const double y = (p == q) ? dia : off;
                c.y3[9 * l + 3 * p + q] = y;
                c.a3[9 * l + 3 * p + q] = (p == q ? 1.0 : 0.0) - 2.0 * R * y;
                c.z3[9 * l + 3 * p + q] = (p == q ? al : 0.0) + be;
            }
        for (int p = 0; p < 3; ++p) {
            const int e = 3 * l + p;
            c.fr_p[e] = P.iperm[3 * net->from[l] + p];
            c.to_p[e] = P.iperm[3 * net->to[l] + p];
            c.g[e] = dia;
            c.alpha[e] = 1.0 - 2.0 * R * dia;
            c.inc_ptr[c.fr_p[e] + 1]++;
            c.inc_ptr[c.to_p[e] + 1]++;
        }
    }
    for (int r = 0; r < n; ++r) {
        c.inc_ptr[r + 1] += c.inc_ptr[r];
        c.gC[r] = 2.0 * net->C[P.perm[r] / 3] / net->dt;
    }
    std::vector<int> fill(c.inc_ptr.begin(), c.inc_ptr.end() - 1);
    for (int e = 0; e < nbr; ++e) {
        c.inc_br[fill[c.fr_p[e]]++] = e;
        c.inc_br[fill[c.to_p[e]]++] = e;
    }
    const int ns = 3 * net->n_src;
    c.src_ptr.assign(n + 1, 0);
    c.samp.assign(ns, 0.0);
    c.sph.assign(ns, 0.0);
    for (int q = 0; q < net->n_src; ++q)
        for (int p = 0; p < 3; ++p) c.src_ptr[P.iperm[3 * net->src_bus[q] + p] + 1]++;
    for (int r = 0; r < n; ++r) c.src_ptr[r + 1] += c.src_ptr[r];
    std::vector<int> sf(c.src_ptr.begin(), c.src_ptr.end() - 1);
    for (int q = 0; q < net->n_src; ++q)
        for (int p = 0; p < 3; ++p) {
            const int r = P.iperm[3 * net->src_bus[q] + p];
            c.samp[sf[r]] = net->amp[q];
            c.sph[sf[r]] = net->phase[q] + p3.shift[p];
            sf[r]++;
        }
}

bool build_team_plan(emt_ctx& c, int R);
void carve_team(emt_ctx& c, Arena& A);
bool build_panel_plan(emt_ctx& c, int R);
void carve_panel(emt_ctx& c, Arena& A);
bool build_level_plan(emt_ctx& c, int R);
void carve_level(emt_ctx& c, Arena& A);
hinv_status upload_level(emt_ctx& c, hipStream_t s);

hinv_status emt_plan3(const emt_network* N, const Phase3& p3, const hinv_tree* T, const hinv_options* o,
                      const emt_cases* C, emt_ctx& c, std::vector<int>& rp, std::vector<int>& ci,
                      std::vector<double>& cv, size_t* bytes);

hinv_status emt_plan(const emt_network* N, const hinv_tree* T, const hinv_options* o, const emt_cases* C,
                     emt_ctx& c, std::vector<int>& rp, std::vector<int>& ci, std::vector<double>& cv, size_t* bytes,
                     const Phase3* p3 = nullptr)
{
    hinv_status st = check_network(N);
    if (st != HINV_OK) return st;
    st = check_options(o, 1);
    if (st != HINV_OK) return st;
    if (o->coupling != HINV_COUPLING_EXACT) return fail(HINV_E_INVALID, "EMT stepping needs coupling = HINV_COUPLING_EXACT");
    c.R = std::max(1, o->max_mod_rank);
    if (p3) return emt_plan3(N, *p3, T, o, C, c, rp, ci, cv, bytes);
    st = check_cases(C, N->n_branch, o->max_mod_rank, c.losses);
    if (st != HINV_OK) return st;
    c.n = N->n_bus;
    c.nbr = N->n_branch;
    c.n_cases = C->n_cases;
    int total_losses = 0;
    for (auto& l : c.losses) total_losses += (int)l.size();
    assemble_csr(N, rp, ci, cv);
    hinv_csr G{N->n_bus, rp.data(), ci.data(), cv.data()};
    st = make_plan(&G, T, c.hc.P);
    if (st != HINV_OK) return st;
    c.hc.opt = *o;
    // scratch columns: one per case per step, one per loss at creation, a full change set later
    c.hc.opt.max_nrhs = std::max(std::max(c.n_cases, c.R), std::max(total_losses, 1));
    prepare_network(c, N);
    Arena A;
    carve_hier(c.hc, A, c.n_cases, c.R, c.hc.opt.max_nrhs);
    carve_emt(c, A, N->n_src);
    // engine
    const int mode = o->kernel_mode;
    const bool fused_prec = (o->prec == HINV_FP64 || o->prec == HINV_FP32);   // the fused engines' formats
    c.team_ok = false;
    if ((mode == 0 || mode == 3) && fused_prec) {
        c.team_nx_cap = 0;
        if (build_team_plan(c, c.R)) {
            c.team_nx_cap = c.TD.NX + 2 * c.R;      // room for the endpoints of later line losses
            c.team_ok = build_team_plan(c, c.R);
        }
        if (!c.table_error.empty()) return fail(HINV_E_DEVICE, "team tables: %s", c.table_error.c_str());
        if (c.team_ok) carve_team(c, A);
    }
    c.panel_ok = false;
    if (((mode == 0 && c.n_cases > 1) || mode == 4) && fused_prec) {
        c.panel_ok = build_panel_plan(c, c.R);
        if (!c.table_error.empty()) return fail(HINV_E_DEVICE, "panel tables: %s", c.table_error.c_str());
        if (c.panel_ok) carve_panel(c, A);
    }
    c.level_ok = false;
    if (((mode == 0 && c.n_cases == 1 && !c.team_ok) || mode == 5) && fused_prec) {
        c.level_nx_cap = 0;
        c.level_ok = build_level_plan(c, c.R);
        if (!c.table_error.empty()) return fail(HINV_E_DEVICE, "level tables: %s", c.table_error.c_str());
        if (c.level_ok) carve_level(c, A);
    }
    const bool fits = run_fits(c.hc.H) && fused_prec;
    if (mode == 5 && !c.level_ok)
        return fail(HINV_E_INVALID, "the level engine needs FP64/FP32, one case, <= 256 leaves of <= %d rows and "
                    "tables that fit LDS", HINV_MAX_LEAF);
    if (mode == 3 && !c.team_ok)
        return fail(HINV_E_INVALID, "the team engine needs FP64/FP32, one case, <= 256 leaves, <= %d coupling "
                    "levels and fitting LDS", kTeamMaxLevels);
    if (mode == 4 && !c.panel_ok)
        return fail(HINV_E_INVALID, "the panel engine needs FP64/FP32, max_mod_rank <= %d, leaves of <= 96 rows, <= 256 leaves and "
                    "coupling columns, and tables that fit LDS", kPanelMaxRank);
    if (mode == 2 && !fits) return fail(HINV_E_INVALID, "the one-workgroup-per-case engine needs FP64/FP32 and a case that fits LDS");
    c.engine = (mode >= 1) ? mode : c.team_ok ? 3 : c.panel_ok ? 4 : c.level_ok ? 5 : fits ? 2 : 1;
    *bytes = A.off + kAlign;
    return HINV_OK;
}

// Three-phase plan: G from assemble_csr3 over rows 3a + p, the bus-level tree with every row in its
// bus's leaf, line losses as groups of three changes (so a case holds max_mod_rank / 3 of them), and
// the per-kernel engine.
hinv_status emt_plan3(const emt_network* N, const Phase3& p3, const hinv_tree* T, const hinv_options* o,
                      const emt_cases* C, emt_ctx& c, std::vector<int>& rp, std::vector<int>& ci,
                      std::vector<double>& cv, size_t* bytes)
{
    if (!(p3.mu >= 0.0 && p3.mu < 0.5)) return fail(HINV_E_INVALID, "mutual ratio %g outside [0, 0.5)", p3.mu);
    for (int p = 0; p < 3; ++p)
        if (!isfinite(p3.shift[p])) return fail(HINV_E_INVALID, "phase shift %d is not finite", p);
    if (o->kernel_mode != 0 && o->kernel_mode != 1 && o->kernel_mode != 2)
        return fail(HINV_E_INVALID, "three-phase networks step on the per-kernel or the one-workgroup-per-case "
                    "engine (kernel_mode 0, 1 or 2)");
    if (!T || !T->parent || !T->bus_leaf) return fail(HINV_E_INVALID, "tree is missing");
    hinv_status st = check_cases(C, N->n_branch, o->max_mod_rank / 3, c.losses);
    if (st != HINV_OK) return st;
    c.ph = 3;
    c.n_lines = N->n_branch;
    c.n = 3 * N->n_bus;
    c.nbr = 3 * N->n_branch;
    c.n_cases = C->n_cases;
    int total_losses = 0;
    for (auto& l : c.losses) total_losses += 3 * (int)l.size();
    assemble_csr3(N, p3.mu, rp, ci, cv);
    hinv_csr G{c.n, rp.data(), ci.data(), cv.data()};
    std::vector<int> leaf3(3 * (size_t)N->n_bus);
    for (int a = 0; a < N->n_bus; ++a)
        for (int p = 0; p < 3; ++p) leaf3[3 * a + p] = T->bus_leaf[a];
    const hinv_tree T3{T->n_nodes, T->parent, leaf3.data()};
    st = make_plan(&G, &T3, c.hc.P);
    if (st != HINV_OK) return st;
    c.hc.opt = *o;
    c.hc.opt.max_nrhs = std::max(std::max(c.n_cases, c.R), std::max(total_losses, 1));
    prepare_network3(c, N, p3);
    Arena A;
    carve_hier(c.hc, A, c.n_cases, c.R, c.hc.opt.max_nrhs);
    carve_emt(c, A, 3 * N->n_src);
    c.team_ok = c.panel_ok = c.level_ok = false;
    const bool fits = run_fits(c.hc.H) && (o->prec == HINV_FP64 || o->prec == HINV_FP32);
    if (o->kernel_mode == 2 && !fits)
        return fail(HINV_E_INVALID, "the one-workgroup-per-case engine needs FP64/FP32 and a case that fits LDS");
    c.engine = (o->kernel_mode == 1 || !fits) ? 1 : 2;
    *bytes = A.off + kAlign;
    return HINV_OK;
}

// ---------------------------------------------------------------------------
// Team plan: per-leaf tables of the team engine (one case; see k_team.hip).
// Bounds check of the team engine's tables (see check_panel_tables).
std::string check_team_tables(const emt_ctx& c)
{
    const Plan& P = c.hc.P;
    const TeamDev& D = c.TD;
    const int L = D.T, H = D.H, Hs = std::max(H, 1), n = c.n, nc = D.nc;
    char buf[256];
    auto bad = [&](const char* fmt, auto... a) {
        snprintf(buf, sizeof buf, fmt, a...);
        return std::string(buf);
    };
    auto mono = [&](const std::vector<int>& a, size_t at, int cnt, int cap) {
        if (a[at] != 0) return false;
        for (int i = 0; i < cnt; ++i)
            if (a[at + i + 1] < a[at + i]) return false;
        return a[at + cnt] <= cap;
    };
    const int npan = (int)P.pan_lo.size();
    for (int l = 0; l < L; ++l) {
        const int lo = c.tw_lo[l], nl = c.tw_nl[l], nx = c.tw_nx[l], nb = c.tw_nb[l], nxu = c.tw_nxu[l], ny = c.tw_ny[l];
        const int ncomb = nl + nx;
        if (lo < 0 || nl < 1 || nl > D.NL || lo + nl > n || nx < 0 || nx > D.NX || nb < 0 || nb > D.NB || nxu < 0 ||
            nxu > nx || ny < 0 || ny > D.NY)
            return bad("leaf %d: counts out of range (lo %d nl %d nx %d nb %d nxu %d ny %d)", l, lo, nl, nx, nb, nxu, ny);
        int xz = 0;
        for (int x = 0; x < nx; ++x) {
            const int r = c.txrow[(size_t)l * D.NX + x];
            if (r < 0 || r >= n || (x > 0 && r <= c.txrow[(size_t)l * D.NX + x - 1]))
                return bad("leaf %d: X row %d (row %d) out of range or order", l, x, r);
            for (int h = 0; h < H; ++h) {
                const size_t i = ((size_t)l * D.NX + x) * H + h;
                const int zo = c.txzo[i], pm = c.txpm[i], pc = c.txpc[i], pp = c.txpan[i];
                if (zo < 0) continue;
                if (pm < 1 || zo + pm > D.XZ || pc < 0 || pc + pm > nc || pp < 0 || pp >= npan)
                    return bad("leaf %d X row %d level %d: Z values (offset %d, %d columns from %d) out of bounds", l,
                               x, h, zo, pm, pc);
                xz = std::max(xz, zo + pm);
            }
        }
        for (int q = 0; q < nxu; ++q) {
            const int x = c.txupd[(size_t)l * D.NX + q];
            if (x < 0 || x >= nx) return bad("leaf %d: updated X row %d out of range", l, x);
            for (int h = 0; h < H; ++h) {
                const int uo = c.tuzo[((size_t)l * D.NX + q) * H + h];
                const int pm = c.txpm[((size_t)l * D.NX + x) * H + h];
                if (uo >= 0 && uo + pm > D.XZU) return bad("leaf %d: updated X row %d Z offset %d beyond %d", l, q, uo, D.XZU);
            }
        }
        for (int h = 0; h < H; ++h) {
            const size_t i = (size_t)l * H + h;
            const int zo = c.tozo[i], pm = c.topm[i], pc = c.topc[i];
            if (zo >= 0 && (pm < 1 || (int64_t)zo + (int64_t)pm * nl > D.ZO || pc < 0 || pc + pm > nc))
                return bad("leaf %d level %d: own Z rows (offset %d, %d columns from %d) out of bounds", l, h, zo, pm, pc);
        }
        for (int g = 0; g < nc; ++g) {
            const int x = c.txpos[(size_t)l * nc + g];
            if (x < 0 || x >= nx || c.txrow[(size_t)l * D.NX + x] != P.col_row[g])
                return bad("leaf %d: column %d maps to X row %d, not its row", l, g, x);
            const int so = c.ttcso[(size_t)l * nc + g], ld = c.ttcld[(size_t)l * nc + g];
            if (so >= 0) {
                const int m = P.node_m[P.col_node[g]];
                if (ld < 2 || (int64_t)so + (int64_t)(m - 1) * ld >= D.sent)
                    return bad("leaf %d: S^-1 row of column %d (offset %d, stride %d) beyond %d entries", l, g, so, ld,
                               D.sent);
            }
        }
        for (int q = 0; q < ny; ++q) {
            const int g = c.tylist[(size_t)l * nc + q];
            if (g < 0 || g >= nc || c.ttcso[(size_t)l * nc + g] < 0)
                return bad("leaf %d: y list entry %d (column %d) has no S^-1 row", l, q, g);
        }
        const size_t rb = (size_t)l * (D.NL + 1);
        if (!mono(c.torp, rb, nl, D.NE) || !mono(c.tiptr, rb, nl, D.NI) || !mono(c.tsptr, rb, nl, D.NS))
            return bad("leaf %d: row pointers not monotone or beyond their tables", l);
        for (int e = 0; e < c.torp[rb + nl]; ++e)
            if (c.tocol[(size_t)l * D.NE + e] < 0 || c.tocol[(size_t)l * D.NE + e] >= ncomb)
                return bad("leaf %d: residual column %d out of range", l, c.tocol[(size_t)l * D.NE + e]);
        for (int e = 0; e < c.tiptr[rb + nl]; ++e)
            if (c.tibr[(size_t)l * D.NI + e] < 0 || c.tibr[(size_t)l * D.NI + e] >= nb)
                return bad("leaf %d: incident branch %d beyond %d branches", l, c.tibr[(size_t)l * D.NI + e], nb);
        for (int q = 0; q < nb; ++q) {
            const size_t i = (size_t)l * D.NB + q;
            if (c.tbglob[i] < 0 || c.tbglob[i] >= c.nbr || c.tbf[i] < 0 || c.tbf[i] >= ncomb || c.tbt[i] < 0 ||
                c.tbt[i] >= ncomb)
                return bad("leaf %d: branch %d (global %d, ends %d %d) out of range", l, q, c.tbglob[i], c.tbf[i], c.tbt[i]);
        }
    }
    for (int g = 0; g < nc; ++g) {
        if (c.taoff[g] < 0 || c.talen[g] < 0 || c.taoff[g] + c.talen[g] > D.nA || c.talo[g] < 0 ||
            c.talo[g] + c.talen[g] > nc)
            return bad("row a_g of column %d (offset %d, columns %d+%d) out of bounds", g, c.taoff[g], c.talo[g], c.talen[g]);
        for (int h = 0; h < Hs; ++h)
            if (c.tcpan[(size_t)g * Hs + h] < -1 || c.tcpan[(size_t)g * Hs + h] >= npan)
                return bad("column %d: panel %d at level %d out of range", g, c.tcpan[(size_t)g * Hs + h], h);
    }
    return std::string();
}

bool build_team_plan(emt_ctx& c, int R)
{
    c.table_error.clear();
    const Plan& P = c.hc.P;
    const int L = (int)P.leaf_lo.size(), H = P.n_levels, n = c.n;
    const int NC = (int)P.col_row.size();
    if (c.n_cases != 1 || L < 1 || L > 256 || H > kTeamMaxLevels) return false;
    // panel of every leaf's rows at every level
    std::vector<int> lpan((size_t)L * std::max(H, 1), -1);
    for (int l = 0; l < L; ++l) {
        for (int k = 0; k < P.anc_stride; ++k) {
            const int t = P.leaf_anc[(size_t)l * P.anc_stride + k];
            if (t < 0) break;
            const int h = P.node_level[t];
            for (int pp = P.node_pan0[t]; pp < P.node_pan0[t] + P.node_npan[t]; ++pp)
                if (P.pan_lo[pp] <= P.leaf_lo[l] && P.leaf_lo[l] < P.pan_lo[pp] + P.pan_n[pp]) lpan[(size_t)l * H + h - 1] = pp;
        }
    }
    std::vector<int> loss_rows;
    for (auto& x : c.losses[0]) {
        loss_rows.push_back(c.fr_p[x.second]);
        loss_rows.push_back(c.to_p[x.second]);
    }
    struct W {
        std::vector<int> xupd;       // X positions of G neighbours of own rows and of line-loss endpoints
        std::vector<int> uzo;        // [xupd.size()*H] their Z values' offsets in LDS, -1: none
        int xzu = 0;
        std::vector<int> xrow, xzo, xpm, xpc, xpan, ozo, opm, opc, opan, xpos, orp, ocol, bglob, bf, bt, bown, iptr, ibr,
            sptr;
        std::vector<double> oval, bg, bal, samp, sph;
        std::vector<int> osrc;       // CSR entry of each oval value, plus one
        int xz = 0, zo = 0;
    };
    std::vector<W> ws(L);
    int XZU = 1;
    int NL = 1, NX = 1, NB = 1, NE = 1, NI = 1, NS = 1, XZ = 1, ZO = 1;
    for (int l = 0; l < L; ++l) {
        W& w = ws[l];
        const int lo = P.leaf_lo[l], nl = P.leaf_n[l];
        auto own = [&](int r) { return r >= lo && r < lo + nl; };
        std::vector<int> X(P.col_row.begin(), P.col_row.end());
        for (int r = lo; r < lo + nl; ++r)
            for (int e = P.rp[r]; e < P.rp[r + 1]; ++e)
                if (!own(P.ci[e])) X.push_back(P.ci[e]);
        for (int r : loss_rows) X.push_back(r);
        std::sort(X.begin(), X.end());
        X.erase(std::unique(X.begin(), X.end()), X.end());
        w.xrow = X;
        auto xpos_of = [&](int row) { return (int)(std::lower_bound(X.begin(), X.end(), row) - X.begin()); };
        auto comb = [&](int row) { return own(row) ? row - lo : nl + xpos_of(row); };
        const int nx = (int)X.size();
        w.xzo.assign((size_t)nx * H, -1); w.xpm.assign((size_t)nx * H, 0); w.xpc.assign((size_t)nx * H, 0);
        w.xpan.assign((size_t)nx * H, -1);
        for (int x = 0; x < nx; ++x) {
            const int lx = P.row_leaf[X[x]];
            for (int h = 1; h <= H; ++h) {
                const int pp = lpan[(size_t)lx * H + h - 1];
                if (pp < 0) continue;
                const size_t i = (size_t)x * H + h - 1;
                w.xpan[i] = pp; w.xzo[i] = w.xz; w.xpm[i] = P.pan_m[pp]; w.xpc[i] = P.pan_col0[pp];
                w.xz += P.pan_m[pp];
            }
        }
        w.ozo.assign(H, -1); w.opm.assign(H, 0); w.opc.assign(H, 0); w.opan.assign(H, -1);
        for (int h = 1; h <= H; ++h) {
            const int pp = lpan[(size_t)l * H + h - 1];
            if (pp < 0) continue;
            w.opan[h - 1] = pp; w.ozo[h - 1] = w.zo; w.opm[h - 1] = P.pan_m[pp]; w.opc[h - 1] = P.pan_col0[pp];
            w.zo += P.pan_m[pp] * nl;
        }
        w.xpos.resize(NC);
        for (int g = 0; g < NC; ++g) w.xpos[g] = xpos_of(P.col_row[g]);
        for (int r = lo; r < lo + nl; ++r)
            for (int e = P.rp[r]; e < P.rp[r + 1]; ++e)
                if (!own(P.ci[e])) w.xupd.push_back(xpos_of(P.ci[e]));
        for (int r : loss_rows) w.xupd.push_back(xpos_of(r));   // the SMW reads endpoints as X rows
        std::sort(w.xupd.begin(), w.xupd.end());
        w.xupd.erase(std::unique(w.xupd.begin(), w.xupd.end()), w.xupd.end());
        w.uzo.assign(w.xupd.size() * (size_t)H, -1);
        for (size_t q = 0; q < w.xupd.size(); ++q)
            for (int h = 0; h < H; ++h) {
                const size_t xi = (size_t)w.xupd[q] * H + h;
                if (w.xzo[xi] < 0) continue;
                w.uzo[q * H + h] = w.xzu;
                w.xzu += w.xpm[xi];
            }
        w.orp.assign(nl + 1, 0);
        for (int r = lo; r < lo + nl; ++r) {
            for (int e = P.rp[r]; e < P.rp[r + 1]; ++e) {
                w.ocol.push_back(comb(P.ci[e]));
                w.oval.push_back(P.cv[e]);
                w.osrc.push_back(e + 1);
            }
            w.orp[r - lo + 1] = (int)w.ocol.size();
        }
        // incident branches (global order of first appearance in the incidence lists)
        std::vector<int> br;
        for (int r = lo; r < lo + nl; ++r)
            for (int q = c.inc_ptr[r]; q < c.inc_ptr[r + 1]; ++q) br.push_back(c.inc_br[q]);
        std::sort(br.begin(), br.end());
        br.erase(std::unique(br.begin(), br.end()), br.end());
        for (int e : br) {
            w.bglob.push_back(e);
            w.bf.push_back(comb(c.fr_p[e]));
            w.bt.push_back(comb(c.to_p[e]));
            w.bown.push_back(own(c.fr_p[e]) ? 1 : 0);
            w.bg.push_back(c.g[e]);
            w.bal.push_back(c.alpha[e]);
        }
        w.iptr.assign(nl + 1, 0);
        w.sptr.assign(nl + 1, 0);
        for (int r = lo; r < lo + nl; ++r) {
            for (int q = c.inc_ptr[r]; q < c.inc_ptr[r + 1]; ++q)
                w.ibr.push_back((int)(std::lower_bound(br.begin(), br.end(), c.inc_br[q]) - br.begin()));
            w.iptr[r - lo + 1] = (int)w.ibr.size();
            for (int q = c.src_ptr[r]; q < c.src_ptr[r + 1]; ++q) {
                w.samp.push_back(c.samp[q]);
                w.sph.push_back(c.sph[q]);
            }
            w.sptr[r - lo + 1] = (int)w.samp.size();
        }
        NL = std::max(NL, nl); NX = std::max(NX, nx); NB = std::max(NB, (int)br.size());
        NE = std::max(NE, (int)w.ocol.size()); NI = std::max(NI, (int)w.ibr.size());
        NS = std::max(NS, (int)w.samp.size()); XZ = std::max(XZ, w.xz); ZO = std::max(ZO, w.zo);
        XZU = std::max(XZU, w.xzu);
    }
    (void)n;
    if (c.team_nx_cap > 0 && NX > c.team_nx_cap) return false;
    TeamDev& D = c.TD;
    D.T = L; D.H = H; D.NL = NL; D.NX = NX; D.NB = NB; D.NE = NE; D.NI = NI; D.NS = NS; D.XZ = XZ; D.ZO = ZO;
    D.XZU = XZU;
    D.nc = NC;
    // y = S^{-1} s is needed only for the columns whose Z values a workgroup applies: the panels of its
    // own rows and of the X rows it updates, at every level.  Only those rows of each node's S^{-1} live
    // in its LDS, as an r x m block per node (r needed rows, leading dimension r + 1 against LDS bank
    // aliasing); the y phase runs over the workgroup's list of needed columns.
    c.ttcso.assign((size_t)L * NC, -1);
    c.ttcld.assign((size_t)L * NC, 0);
    c.tylist.assign((size_t)L * NC, 0);
    c.tw_ny.assign(L, 0);
    {
        int64_t sent = 1;
        int ny_max = 1;
        std::vector<char> need(NC);
        for (int l = 0; l < L; ++l) {
            const W& w = ws[l];
            std::fill(need.begin(), need.end(), 0);
            for (int h = 0; h < H; ++h)
                if (w.ozo[h] >= 0)
                    for (int j = 0; j < w.opm[h]; ++j) need[w.opc[h] + j] = 1;
            for (int x : w.xupd)
                for (int h = 0; h < H; ++h) {
                    const size_t xi = (size_t)x * H + h;
                    if (w.xzo[xi] < 0) continue;
                    for (int j = 0; j < w.xpm[xi]; ++j) need[w.xpc[xi] + j] = 1;
                }
            int64_t off = 0;
            int ny = 0;
            for (size_t t = 0; t < P.node_m.size(); ++t) {
                const int m = P.node_m[t], c0 = P.node_col0[t];
                int r = 0;
                for (int q = 0; q < m; ++q) r += need[c0 + q];
                if (r == 0) continue;
                int slot = 0;
                for (int q = 0; q < m; ++q) {
                    if (!need[c0 + q]) continue;
                    c.ttcso[(size_t)l * NC + c0 + q] = (int)(off + slot++);
                    c.ttcld[(size_t)l * NC + c0 + q] = r + 1;
                    c.tylist[(size_t)l * NC + ny++] = c0 + q;
                }
                off += (int64_t)(r + 1) * m;
            }
            c.tw_ny[l] = ny;
            sent = std::max(sent, off);
            ny_max = std::max(ny_max, ny);
        }
        D.sent = (int)sent;
        D.NY = ny_max;
    }
    // rows a_g of the two-phase coupling levels (values from launch_team_acoef): the panel of the
    // column's row at every lower level, and the columns a_g can reach, as one range per column
    {
        const int Hs = std::max(H, 1);
        c.tcpan.assign((size_t)NC * Hs, -1);
        c.taoff.assign(NC, 0); c.talo.assign(NC, 0); c.talen.assign(NC, 0);
        // covering ranges [lo, hi] of the columns that s_g (off its own column) and y_g depend on
        std::vector<int> alo_(NC, INT32_MAX), ahi_(NC, -1), blo_(NC, INT32_MAX), bhi_(NC, -1);
        for (int h = 1; h <= H; ++h) {
            for (int g = P.lvl_col[h - 1]; g < P.lvl_col[h]; ++g) {
                const int lf = P.row_leaf[P.col_row[g]];
                for (int hh = 1; hh < h; ++hh) {
                    const int pp = lpan[(size_t)lf * H + hh - 1];
                    c.tcpan[(size_t)g * Hs + hh - 1] = pp;
                    if (pp < 0) continue;
                    for (int j = 0; j < P.pan_m[pp]; ++j) {
                        const int gp = P.pan_col0[pp] + j;
                        alo_[g] = std::min(alo_[g], blo_[gp]);
                        ahi_[g] = std::max(ahi_[g], bhi_[gp]);
                    }
                }
            }
            for (int g = P.lvl_col[h - 1]; g < P.lvl_col[h]; ++g) {
                const int t = P.col_node[g], c0 = P.node_col0[t], m = P.node_m[t];
                blo_[g] = c0;
                bhi_[g] = c0 + m - 1;
                for (int p = 0; p < m; ++p) {
                    blo_[g] = std::min(blo_[g], alo_[c0 + p]);
                    bhi_[g] = std::max(bhi_[g], ahi_[c0 + p]);
                }
            }
        }
        int na = 0;
        for (int g = 0; g < NC; ++g) {
            c.taoff[g] = na;
            c.talo[g] = ahi_[g] < 0 ? 0 : alo_[g];
            c.talen[g] = ahi_[g] < 0 ? 0 : ahi_[g] - alo_[g] + 1;
            na += c.talen[g];
        }
        D.nA = std::max(na, 1);
    }
    if (team_lds_bytes(D, c.hc.H, R, c.hc.opt.prec, c.hc.opt.warm_start ? 1 : 0) > 160 * 1024) return false;
    const int Hs = std::max(H, 1);
    (void)Hs;
    auto flat = [&](std::vector<int>& dst, size_t stride, auto get) {
        dst.assign((size_t)L * stride, 0);
        for (int l = 0; l < L; ++l) {
            const std::vector<int>& src = get(ws[l]);
            std::copy(src.begin(), src.end(), dst.begin() + (size_t)l * stride);
        }
    };
    auto flatd = [&](std::vector<double>& dst, size_t stride, auto get) {
        dst.assign((size_t)L * stride, 0.0);
        for (int l = 0; l < L; ++l) {
            const std::vector<double>& src = get(ws[l]);
            std::copy(src.begin(), src.end(), dst.begin() + (size_t)l * stride);
        }
    };
    const int NXc = c.team_nx_cap > 0 ? c.team_nx_cap : NX;
    c.tw_lo = P.leaf_lo; c.tw_nl = P.leaf_n;
    c.tw_nx.resize(L); c.tw_nb.resize(L); c.tw_nxu.resize(L);
    for (int l = 0; l < L; ++l) {
        c.tw_nx[l] = (int)ws[l].xrow.size(); c.tw_nb[l] = (int)ws[l].bglob.size(); c.tw_nxu[l] = (int)ws[l].xupd.size();
    }
    // X-row tables use the capacity stride so that a later rebuild fits the carve
    flat(c.txrow, NXc, [](W& w) -> std::vector<int>& { return w.xrow; });
    flat(c.txupd, NXc, [](W& w) -> std::vector<int>& { return w.xupd; });
    flat(c.tuzo, (size_t)NXc * H, [](W& w) -> std::vector<int>& { return w.uzo; });
    flat(c.txzo, (size_t)NXc * H, [](W& w) -> std::vector<int>& { return w.xzo; });
    flat(c.txpm, (size_t)NXc * H, [](W& w) -> std::vector<int>& { return w.xpm; });
    flat(c.txpc, (size_t)NXc * H, [](W& w) -> std::vector<int>& { return w.xpc; });
    flat(c.txpan, (size_t)NXc * H, [](W& w) -> std::vector<int>& { return w.xpan; });
    flat(c.tozo, H, [](W& w) -> std::vector<int>& { return w.ozo; });
    flat(c.topm, H, [](W& w) -> std::vector<int>& { return w.opm; });
    flat(c.topc, H, [](W& w) -> std::vector<int>& { return w.opc; });
    flat(c.topan, H, [](W& w) -> std::vector<int>& { return w.opan; });
    flat(c.txpos, NC, [](W& w) -> std::vector<int>& { return w.xpos; });
    flat(c.torp, NL + 1, [](W& w) -> std::vector<int>& { return w.orp; });
    flat(c.tocol, NE, [](W& w) -> std::vector<int>& { return w.ocol; });
    flat(c.tbglob, NB, [](W& w) -> std::vector<int>& { return w.bglob; });
    flat(c.tbf, NB, [](W& w) -> std::vector<int>& { return w.bf; });
    flat(c.tbt, NB, [](W& w) -> std::vector<int>& { return w.bt; });
    flat(c.tbown, NB, [](W& w) -> std::vector<int>& { return w.bown; });
    flat(c.tiptr, NL + 1, [](W& w) -> std::vector<int>& { return w.iptr; });
    flat(c.tibr, NI, [](W& w) -> std::vector<int>& { return w.ibr; });
    flat(c.tsptr, NL + 1, [](W& w) -> std::vector<int>& { return w.sptr; });
    flatd(c.toval, NE, [](W& w) -> std::vector<double>& { return w.oval; });
    flat(c.tosrc, NE, [](W& w) -> std::vector<int>& { return w.osrc; });
    flatd(c.tbg, NB, [](W& w) -> std::vector<double>& { return w.bg; });
    flatd(c.tbal, NB, [](W& w) -> std::vector<double>& { return w.bal; });
    flatd(c.tsamp, NS, [](W& w) -> std::vector<double>& { return w.samp; });
    flatd(c.tsph, NS, [](W& w) -> std::vector<double>& { return w.sph; });
    D.NX = NXc;   // strides of the device tables (and the LDS layout)
    if (team_lds_bytes(D, c.hc.H, R, c.hc.opt.prec, c.hc.opt.warm_start ? 1 : 0) > 160 * 1024) return false;
    c.table_error = check_team_tables(c);
    return c.table_error.empty();
}

// Workspace for the team tables (sizes from the current plan, X rows with capacity).
void carve_team(emt_ctx& c, Arena& A)
{
    TeamDev& D = c.TD;
    const int64_t L = D.T, H = D.H;
    auto ti = [&](size_t cnt) { return A.take<int>((int64_t)cnt); };
    auto td = [&](size_t cnt) { return A.take<double>((int64_t)cnt); };
    D.w_lo = ti(L); D.w_nl = ti(L); D.w_nx = ti(L); D.w_nb = ti(L);
    D.w_nxu = ti(L); D.xupd = ti(L * D.NX); D.uzo = ti(L * D.NX * H);
    D.xrow = ti(L * D.NX); D.xzo = ti(L * D.NX * H); D.xpm = ti(L * D.NX * H); D.xpc = ti(L * D.NX * H);
    D.xpan = ti(L * D.NX * H);
    D.ozo = ti(L * H); D.opm = ti(L * H); D.opc = ti(L * H); D.opan = ti(L * H);
    D.xpos = ti(L * D.nc);
    D.orp = ti(L * (D.NL + 1)); D.ocol = ti(L * D.NE); D.oval = td(L * D.NE);
    D.bglob = ti(L * D.NB); D.bf = ti(L * D.NB); D.bt = ti(L * D.NB); D.bown = ti(L * D.NB);
    D.bg = td(L * D.NB); D.bal = td(L * D.NB);
    D.iptr = ti(L * (D.NL + 1)); D.ibr = ti(L * D.NI);
    D.sptr = ti(L * (D.NL + 1)); D.samp = td(L * D.NS); D.sph = td(L * D.NS);
    D.sync = A.take<unsigned int>(L);
    D.csop = ti((size_t)L * D.nc); D.cld = ti((size_t)L * D.nc); D.ylist = ti((size_t)L * D.nc); D.w_ny = ti(L);
    D.X0 = td(2 * (size_t)c.n);
    D.VM = td(2 * L);
    D.aoff = ti(D.nc); D.alo = ti(D.nc); D.alen = ti(D.nc);
    D.cpan = ti((size_t)D.nc * std::max<int64_t>(H, 1));
    D.acoef = td(D.nA);
    D.acoef32 = A.take<float>(D.nA);
    D.am = td((size_t)D.nc * D.nc);
    D.bm = td((size_t)D.nc * D.nc);
}

// ---------------------------------------------------------------------------
// Bounds check of the panel engine's tables against the sizes the kernel and its LDS layout assume:
// every index a workgroup uses to address LDS, its registers' item ranges or a global array is
// within the region it addresses.  Returns the first violation (empty: none).  Host only, so it runs
// in emt_workspace_size as well as before every upload.
std::string check_panel_tables(const emt_ctx& c, int R)
{
    const Plan& P = c.hc.P;
    const PanelDev& D = c.PD;
    const int L = D.T, Hs = std::max(D.H, 1), n = c.n, nc = D.nc;
    char buf[256];
    auto bad = [&](const char* fmt, auto... a) {
        snprintf(buf, sizeof buf, fmt, a...);
        return std::string(buf);
    };
    int64_t zsize = 0;
    for (size_t p = 0; p < P.pan_zoff.size(); ++p) zsize = std::max(zsize, P.pan_zoff[p] + (int64_t)P.pan_n[p] * P.pan_m[p]);
    if (D.NL < 1 || D.NL > kPanelMaxLeaf || D.NLp % 16 || D.NLp < D.NL || D.NX > kPanelMaxX || nc > kPanelMaxCols ||
        D.ncp < nc || D.ncp % 4 || D.NB * kPanelCases > 6 * kPanelWaves * 64 || R > kPanelMaxRank ||
        L * std::max(R, 1) * kPanelCases > kPanelWaves * 64 || D.NY % 16 || D.MF % 64)
        return bad("panel dimensions NL %d NLp %d NX %d NB %d nc %d ncp %d NY %d MF %d outside the kernel's limits",
                   D.NL, D.NLp, D.NX, D.NB, nc, D.ncp, D.NY, D.MF);
    auto mono = [&](const std::vector<int>& a, size_t at, int cnt, int cap) {
        if (a[at] != 0) return false;
        for (int i = 0; i < cnt; ++i)
            if (a[at + i + 1] < a[at + i]) return false;
        return a[at + cnt] <= cap;
    };
    for (int l = 0; l < L; ++l) {
        const int lo = c.tw_lo[l], nl = c.tw_nl[l], nx = c.pw_nx[l], nb = c.tw_nb[l], ny = c.pw_ny[l],
                  nt = c.pw_nt[l], np = c.pw_np[l], nxz = c.pw_xz[l];
        const int ncomb = nl + nx;
        if (lo < 0 || nl < 1 || nl > D.NL || lo + nl > n || nx < 0 || nx > D.NX || nb < 0 || nb > D.NB || ny < 0 ||
            ny > D.NY || ny % 16 || nt < 0 || nt > D.NT || nt > kPanelWaves * kPanelYTasksPerWave || np < 0 ||
            np > D.NP || nxz < 0 || nxz > D.XZ || ncomb >= (1 << 16))
            return bad("leaf %d: counts out of range (lo %d nl %d nx %d nb %d ny %d nt %d np %d xz %d)", l, lo, nl, nx,
                       nb, ny, nt, np, nxz);
        for (int x = 0; x < nx; ++x) {
            const int r = c.pxrow[(size_t)l * D.NX + x], g = c.pxcol[(size_t)l * D.NX + x];
            if (r < 0 || r >= n || (r >= lo && r < lo + nl) || g < 0 || g >= nc || P.col_row[g] != r)
                return bad("leaf %d: X row %d (row %d, column %d) invalid", l, x, r, g);
        }
        for (int h = 0; h < Hs; ++h) {
            const size_t i = (size_t)l * Hs + h;
            const int zo = c.tozo[i], pm = c.topm[i], ps = c.topc[i];
            if (zo >= 0 && (pm < 1 || (int64_t)zo + (int64_t)pm * nl > D.ZO || ps < 0 || ps + pm > ny))
                return bad("leaf %d level %d: own Z rows (offset %d, %d columns, slot %d) out of bounds", l, h, zo, pm, ps);
            for (int x = 0; x < nx; ++x) {
                const size_t j = ((size_t)l * D.NX + x) * Hs + h;
                const int xo = c.pxzo[j], xm = c.pxpm[j], xs = c.pxps[j];
                if (xo >= 0 && (xm < 1 || xo + xm > nxz || xs < 0 || xs + xm > ny))
                    return bad("leaf %d X row %d level %d: Z values (offset %d, %d columns, slot %d) out of bounds", l, x,
                               h, xo, xm, xs);
            }
        }
        for (int i = 0; i < nxz; ++i) {
            const int z = c.pxzsrc[(size_t)l * D.XZ + i];
            if (z < 0 || z >= zsize) return bad("leaf %d: X-row Z source %d outside the Z panels", l, z);
        }
        const size_t rb = (size_t)l * (D.NL + 1);
        if (!mono(c.torp, rb, nl, D.NE) || !mono(c.tiptr, rb, nl, D.NI) || !mono(c.tsptr, rb, nl, D.NS))
            return bad("leaf %d: row pointers not monotone or beyond their tables", l);
        for (int e = 0; e < c.torp[rb + nl]; ++e)
            if (c.tocol[(size_t)l * D.NE + e] < 0 || c.tocol[(size_t)l * D.NE + e] >= ncomb)
                return bad("leaf %d: residual column %d out of range", l, c.tocol[(size_t)l * D.NE + e]);
        for (int e = 0; e < c.tiptr[rb + nl]; ++e) {
            const int v = c.tibr[(size_t)l * D.NI + e], lb = v >= 0 ? v : ~v;
            if (lb >= nb) return bad("leaf %d: incident branch %d beyond %d branches", l, lb, nb);
        }
        for (int q = 0; q < nb; ++q) {
            const size_t i = (size_t)l * D.NB + q;
            const int f = c.phbft[i] & 0xffff, t = c.phbft[i] >> 16;
            if (c.tbglob[i] < 0 || c.tbglob[i] >= c.nbr || f >= ncomb || t >= ncomb || f != c.tbf[i] || t != c.tbt[i])
                return bad("leaf %d: branch %d (global %d, ends %d %d) out of range", l, q, c.tbglob[i], f, t);
        }
        for (int q = 0; q < np; ++q) {
            const int r = c.ppubr[(size_t)l * D.NP + q], g = c.ppubg[(size_t)l * D.NP + q];
            if (r < 0 || r >= nl || g < 0 || g >= nc) return bad("leaf %d: published pair (%d, %d) out of range", l, r, g);
        }
        for (int q = 0; q < ny; ++q) {
            const int g = c.pyslot[(size_t)l * D.NY + q];
            if (g < -1 || g >= nc) return bad("leaf %d: y slot %d holds column %d", l, q, g);
        }
        const int ntile = ny / 16;
        if (c.pttp[(size_t)l * (D.NY / 16 + 1)] != 0 || c.pttp[(size_t)l * (D.NY / 16 + 1) + ntile] != nt)
            return bad("leaf %d: task pointers do not cover the %d tasks", l, nt);
        for (int t = 0; t < ntile; ++t)
            if (c.pttp[(size_t)l * (D.NY / 16 + 1) + t + 1] < c.pttp[(size_t)l * (D.NY / 16 + 1) + t])
                return bad("leaf %d: task pointers not monotone", l);
        std::vector<int> seen(nt, 0);
        for (int t = 0; t < nt; ++t) {
            const size_t i = (size_t)l * D.NT + t;
            const int k0 = c.ptk0[i], nk = c.ptnk[i], fo = c.ptfo[i], tile = c.pttile[i], tl = c.pttl[i];
            if (k0 < 0 || nk < 1 || (k0 + nk) * 4 > D.ncp || fo < 0 || fo % 64 || fo + nk * 64 > D.MF || tile < 0 ||
                tile >= ntile || tl < 0 || tl >= nt)
                return bad("leaf %d: y task %d (k %d+%d, fragments %d, tile %d) out of bounds", l, t, k0, nk, fo, tile);
        }
        for (int w = 0; w < kPanelWaves * kPanelYTasksPerWave; ++w) {
            const int t = c.pwtask[(size_t)l * kPanelWaves * kPanelYTasksPerWave + w];
            if (t < -1 || t >= nt || (t >= 0 && seen[t]++)) return bad("leaf %d: wavefront task slot %d holds %d", l, w, t);
        }
        for (int t = 0; t < nt; ++t)
            if (!seen[t]) return bad("leaf %d: y task %d has no wavefront", l, t);
    }
    for (size_t i = 0; i < c.plpa.size(); ++i) {
        const int tl = (int)(i / ((size_t)kPanelCases * R)) % L;
        const int ncomb = c.tw_nl[tl] + c.pw_nx[tl];
        if (c.plpa[i] < -1 || c.plpa[i] >= ncomb || c.plpb[i] < -1 || c.plpb[i] >= ncomb)
            return bad("change endpoint rows (%d, %d) out of range", c.plpa[i], c.plpb[i]);
    }
    return std::string();
}

// ---------------------------------------------------------------------------
// Panel plan: per-leaf tables (shared with the team layout's per-leaf vectors;
// an EMT handle uses one of the two engines), per (team, leaf) X rows and
// change endpoints, and the coupling columns' lower-level Z rows.
bool build_panel_plan(emt_ctx& c, int R)
{
    c.table_error.clear();
    const Plan& P = c.hc.P;
    const int L = (int)P.leaf_lo.size(), H = P.n_levels, NC = (int)P.col_row.size();
    // one thread per (workgroup, change, case) gathers the shares of u^T x
    if (R > kPanelMaxRank || L < 1 || L * std::max(R, 1) * kPanelCases > kPanelWaves * 64 || NC > kPanelMaxCols || H < 0)
        return false;
    const int n_teams = (c.n_cases + kPanelCases - 1) / kPanelCases;
    const int Hs = std::max(H, 1);
    std::vector<int> lpan((size_t)L * Hs, -1);       // panel of leaf l's rows at level h
    for (int l = 0; l < L; ++l) {
        for (int k = 0; k < P.anc_stride; ++k) {
            const int t = P.leaf_anc[(size_t)l * P.anc_stride + k];
            if (t < 0) break;
            const int h = P.node_level[t];
            for (int pp = P.node_pan0[t]; pp < P.node_pan0[t] + P.node_npan[t]; ++pp)
                if (P.pan_lo[pp] <= P.leaf_lo[l] && P.leaf_lo[l] < P.pan_lo[pp] + P.pan_n[pp]) lpan[(size_t)l * Hs + h - 1] = pp;
        }
    }
    // the map y = M u: the panel of each column's row at every lower level (for its device build), and the
    // columns each y depends on, as one covering range per column (bottom-up, as the levels compose)
    c.pcpan.assign((size_t)NC * Hs, -1);
    std::vector<int> blo(NC, 0), bhi(NC, -1);
    {
        std::vector<int> alo(NC, INT32_MAX), ahi(NC, -1);
        for (int h = 1; h <= H; ++h) {
            for (int g = P.lvl_col[h - 1]; g < P.lvl_col[h]; ++g) {
                const int lf = P.row_leaf[P.col_row[g]];
                for (int hh = 1; hh < h; ++hh) {
                    const int pp = lpan[(size_t)lf * Hs + hh - 1];
                    c.pcpan[(size_t)g * Hs + hh - 1] = pp;
                    if (pp < 0) continue;
                    for (int j = 0; j < P.pan_m[pp]; ++j) {
                        const int gp = P.pan_col0[pp] + j;
                        alo[g] = std::min(alo[g], blo[gp]);
                        ahi[g] = std::max(ahi[g], bhi[gp]);
                    }
                }
            }
            for (int g = P.lvl_col[h - 1]; g < P.lvl_col[h]; ++g) {
                const int t = P.col_node[g], c0 = P.node_col0[t], m = P.node_m[t];
                blo[g] = c0;
                bhi[g] = c0 + m - 1;
                for (int p = 0; p < m; ++p) {
                    if (ahi[c0 + p] < 0) continue;
                    blo[g] = std::min(blo[g], alo[c0 + p]);
                    bhi[g] = std::max(bhi[g], ahi[c0 + p]);
                }
            }
        }
    }
    std::vector<int> row_col(c.n, -1);               // a coupling column of each row
    for (int g = NC - 1; g >= 0; --g) row_col[P.col_row[g]] = g;
    // per leaf: X rows (neighbours through G in other leaves), own Z panels, CSR rows, branches, sources,
    // published columns, y slots and tasks
    struct W {
        std::vector<int> fx, xcol, ozo, opm, ops, opan, orp, ocol, bglob, bf, bt, bown, iptr, ibr, sptr, pubr, pubg;
        std::vector<int> xzo, xpm, xps, xpan, yslot, tk0, tnk, tfo, ttile, ttp, ttl, wtask, ibrs, hbft, xzsrc;
        std::vector<double> oval, bg, bal, samp, sph;
        std::vector<int> osrc;       // CSR entry of each oval value, plus one
        int zo = 0, xz = 0, mf = 0;
    };
    std::vector<W> ws(L);
    int NL = 1, NB = 1, NE = 1, NI = 1, NS = 1, ZO = 1, NX = 1, XZ = 1, NY = 16, NT = 1, MF = 64, NP = 1;
    for (int l = 0; l < L; ++l) {
        W& w = ws[l];
        const int lo = P.leaf_lo[l], nl = P.leaf_n[l];
        auto own = [&](int r) { return r >= lo && r < lo + nl; };
        for (int r = lo; r < lo + nl; ++r)
            for (int e = P.rp[r]; e < P.rp[r + 1]; ++e)
                if (!own(P.ci[e])) w.fx.push_back(P.ci[e]);
        std::sort(w.fx.begin(), w.fx.end());
        w.fx.erase(std::unique(w.fx.begin(), w.fx.end()), w.fx.end());
        for (int x : w.fx) {
            if (row_col[x] < 0) return false;        // a neighbour in another leaf is the end of a cut line
            w.xcol.push_back(row_col[x]);
        }
        auto comb = [&](int row) {
            return own(row) ? row - lo : nl + (int)(std::lower_bound(w.fx.begin(), w.fx.end(), row) - w.fx.begin());
        };
        // columns whose y this workgroup applies: its own rows' panels and its X rows' panels
        std::vector<int> need;
        for (int h = 1; h <= H; ++h) {
            const int pp = lpan[(size_t)l * Hs + h - 1];
            if (pp >= 0)
                for (int q = 0; q < P.pan_m[pp]; ++q) need.push_back(P.pan_col0[pp] + q);
            for (int x : w.fx) {
                const int px = lpan[(size_t)P.row_leaf[x] * Hs + h - 1];
                if (px >= 0)
                    for (int q = 0; q < P.pan_m[px]; ++q) need.push_back(P.pan_col0[px] + q);
            }
        }
        std::sort(need.begin(), need.end());
        need.erase(std::unique(need.begin(), need.end()), need.end());
        // slots: columns with the same dependency range together, each range group padded to 16-row tiles
        std::stable_sort(need.begin(), need.end(), [&](int a, int b) {
            return blo[a] != blo[b] ? blo[a] < blo[b] : bhi[a] != bhi[b] ? bhi[a] < bhi[b] : a < b;
        });
        std::vector<int> slot_of(NC, -1);
        for (size_t q = 0; q < need.size();) {
            size_t e = q;
            while (e < need.size() && blo[need[e]] == blo[need[q]] && bhi[need[e]] == bhi[need[q]]) ++e;
            for (size_t k = q; k < e; ++k) {
                slot_of[need[k]] = (int)w.yslot.size();
                w.yslot.push_back(need[k]);
            }
            while (w.yslot.size() % 16) w.yslot.push_back(-1);
            q = e;
        }
        // tasks: a tile's k-steps (those of its range group) in ceil(k-steps / kPanelYChain) near-equal
        // chains, a split that depends on the range alone
        const int ntile = (int)w.yslot.size() / 16;
        w.ttp.assign(ntile + 1, 0);
        for (int t = 0; t < ntile; ++t) {
            int g0 = -1;
            for (int k = 0; k < 16 && g0 < 0; ++k) g0 = w.yslot[t * 16 + k];
            const int kb = blo[g0] / 4, ke = bhi[g0] / 4 + 1, nk = ke - kb;
            const int nsplit = (nk + kPanelYChain - 1) / kPanelYChain;
            for (int q = 0; q < nsplit; ++q) {
                const int a = kb + (int)((int64_t)q * nk / nsplit), b = kb + (int)((int64_t)(q + 1) * nk / nsplit);
                w.ttl.push_back((int)w.tk0.size());
                w.tk0.push_back(a);
                w.tnk.push_back(b - a);
                w.tfo.push_back(w.mf);
                w.ttile.push_back(t);
                w.mf += (b - a) * 64;
            }
            w.ttp[t + 1] = (int)w.ttl.size();
        }
        // tasks onto wavefronts: largest first, each to the least loaded SIMD (wavefront w runs on SIMD w % 4)
        // and there to its least loaded wavefront with a free place
        {
            const int nt = (int)w.tk0.size();
            if (nt > kPanelWaves * kPanelYTasksPerWave) return false;
            std::vector<int> ord(nt);
            for (int t = 0; t < nt; ++t) ord[t] = t;
            std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return w.tnk[a] > w.tnk[b]; });
            std::vector<int> load(kPanelWaves, 0), used(kPanelWaves, 0), sload(4, 0);
            w.wtask.assign(kPanelWaves * kPanelYTasksPerWave, -1);
            for (int t : ord) {
                int best = -1;
                for (int q = 0; q < kPanelWaves; ++q) {
                    if (used[q] >= kPanelYTasksPerWave) continue;
                    if (best < 0 || sload[q % 4] < sload[best % 4] ||
                        (sload[q % 4] == sload[best % 4] && load[q] < load[best])) best = q;
                }
                w.wtask[best * kPanelYTasksPerWave + used[best]++] = t;
                load[best] += w.tnk[t];
                sload[best % 4] += w.tnk[t];
            }
        }
        w.ozo.assign(Hs, -1); w.opm.assign(Hs, 0); w.ops.assign(Hs, 0); w.opan.assign(Hs, -1);
        for (int h = 1; h <= H; ++h) {
            const int pp = lpan[(size_t)l * Hs + h - 1];
            if (pp < 0) continue;
            w.opan[h - 1] = pp; w.ozo[h - 1] = w.zo; w.opm[h - 1] = P.pan_m[pp];
            w.ops[h - 1] = slot_of[P.pan_col0[pp]];
            w.zo += P.pan_m[pp] * nl;
        }
        w.xzo.assign((size_t)w.fx.size() * Hs, -1); w.xpm.assign((size_t)w.fx.size() * Hs, 0);
        w.xps.assign((size_t)w.fx.size() * Hs, 0); w.xpan.assign((size_t)w.fx.size() * Hs, -1);
        for (size_t x = 0; x < w.fx.size(); ++x) {
            const int lx = P.row_leaf[w.fx[x]];
            for (int h = 1; h <= H; ++h) {
                const int pp = lpan[(size_t)lx * Hs + h - 1];
                if (pp < 0) continue;
                const size_t i = x * Hs + h - 1;
                w.xzo[i] = w.xz; w.xpm[i] = P.pan_m[pp]; w.xps[i] = slot_of[P.pan_col0[pp]]; w.xpan[i] = pp;
                for (int j = 0; j < P.pan_m[pp]; ++j)
                    w.xzsrc.push_back((int)(P.pan_zoff[pp] + (w.fx[x] - P.pan_lo[pp]) + (int64_t)j * P.pan_n[pp]));
                w.xz += P.pan_m[pp];
            }
        }
        for (int g = 0; g < NC; ++g)
            if (own(P.col_row[g])) {
                w.pubr.push_back(P.col_row[g] - lo);
                w.pubg.push_back(g);
            }
        w.orp.assign(nl + 1, 0);
        for (int r = lo; r < lo + nl; ++r) {
            for (int e = P.rp[r]; e < P.rp[r + 1]; ++e) {
                w.ocol.push_back(comb(P.ci[e]));
                w.oval.push_back(P.cv[e]);
                w.osrc.push_back(e + 1);
            }
            w.orp[r - lo + 1] = (int)w.ocol.size();
        }
        std::vector<int> br;
        for (int r = lo; r < lo + nl; ++r)
            for (int q = c.inc_ptr[r]; q < c.inc_ptr[r + 1]; ++q) br.push_back(c.inc_br[q]);
        std::sort(br.begin(), br.end());
        br.erase(std::unique(br.begin(), br.end()), br.end());
        for (int e : br) {
            w.bglob.push_back(e);
            w.bf.push_back(comb(c.fr_p[e]));
            w.bt.push_back(comb(c.to_p[e]));
            w.hbft.push_back(w.bf.back() | (w.bt.back() << 16));
            w.bown.push_back(own(c.fr_p[e]) ? 1 : 0);
            w.bg.push_back(c.g[e]);
            w.bal.push_back(c.alpha[e]);
        }
        w.iptr.assign(nl + 1, 0);
        w.sptr.assign(nl + 1, 0);
        for (int r = lo; r < lo + nl; ++r) {
            for (int q = c.inc_ptr[r]; q < c.inc_ptr[r + 1]; ++q) {
                const int lb = (int)(std::lower_bound(br.begin(), br.end(), c.inc_br[q]) - br.begin());
                w.ibr.push_back(lb);
                w.ibrs.push_back(w.bf[lb] == r - lo ? lb : ~lb);
            }
            w.iptr[r - lo + 1] = (int)w.ibr.size();
            for (int q = c.src_ptr[r]; q < c.src_ptr[r + 1]; ++q) {
                w.samp.push_back(c.samp[q]);
                w.sph.push_back(c.sph[q]);
            }
            w.sptr[r - lo + 1] = (int)w.samp.size();
        }
        NL = std::max(NL, nl); NB = std::max(NB, (int)br.size());
        NE = std::max(NE, (int)w.ocol.size()); NI = std::max(NI, (int)w.ibr.size());
        NS = std::max(NS, (int)w.samp.size()); ZO = std::max(ZO, w.zo);
        NX = std::max(NX, (int)w.fx.size()); XZ = std::max(XZ, w.xz);
        NY = std::max(NY, (int)w.yslot.size()); NT = std::max(NT, (int)w.tk0.size());
        MF = std::max(MF, w.mf); NP = std::max(NP, (int)w.pubg.size());
    }
    // history items per thread (kernel: 6 of 512 threads' (branch, case) items); combined indices in 16 bits
    if (NX > kPanelMaxX || NL > kPanelMaxLeaf || NB * kPanelCases > 6 * kPanelWaves * 64) return false;
    // per (team, leaf): the combined index of each change's endpoints where it is a row of the workgroup
    // (a change's other endpoint is then a neighbour through G, hence a row too; the refinement residual
    // takes the change's term on such rows), -1 elsewhere
    std::vector<int> lpa((size_t)n_teams * L * kPanelCases * R, -1), lpb((size_t)n_teams * L * kPanelCases * R, -1);
    for (int tm = 0; tm < n_teams; ++tm) {
        for (int l = 0; l < L; ++l) {
            const W& w = ws[l];
            const int lo = P.leaf_lo[l], nl = P.leaf_n[l];
            auto comb = [&](int row) {
                if (row >= lo && row < lo + nl) return row - lo;
                auto it = std::lower_bound(w.fx.begin(), w.fx.end(), row);
                return (it != w.fx.end() && *it == row) ? nl + (int)(it - w.fx.begin()) : -1;
            };
            for (int cc = 0; cc < kPanelCases; ++cc) {
                const int k = tm * kPanelCases + cc;
                if (k >= c.n_cases) break;
                const auto& Lk = c.losses[k];
                for (size_t j = 0; j < Lk.size() && (int)j < R; ++j) {
                    const int a = comb(c.fr_p[Lk[j].second]), b = comb(c.to_p[Lk[j].second]);
                    const bool own_a = a >= 0 && a < nl, own_b = b >= 0 && b < nl;
                    if ((own_a && b < 0) || (own_b && a < 0)) return false;
                    const size_t o = (((size_t)tm * L + l) * kPanelCases + cc) * R + j;
                    lpa[o] = a;
                    lpb[o] = b;
                }
            }
        }
    }
    std::vector<int> hlost((size_t)n_teams * L * NB * kPanelCases, 0x7fffffff);
    for (int tm = 0; tm < n_teams; ++tm)
        for (int cc = 0; cc < kPanelCases; ++cc) {
            const int k = tm * kPanelCases + cc;
            if (k >= c.n_cases) break;
            for (const auto& ls : c.losses[k])
                for (int l = 0; l < L; ++l) {
                    const auto& bgl = ws[l].bglob;
                    const auto it = std::lower_bound(bgl.begin(), bgl.end(), ls.second);
                    if (it == bgl.end() || *it != ls.second) continue;
                    int& v = hlost[(((size_t)tm * L + l) * NB + (it - bgl.begin())) * kPanelCases + cc];
                    v = std::min(v, ls.first);
                }
        }
    PanelDev& D = c.PD;
    D.T = L; D.H = H; D.NL = NL; D.NLp = (NL + 15) / 16 * 16; D.NX = NX; D.NB = NB; D.NE = NE;
    D.NI = NI; D.NS = NS; D.XZ = XZ; D.ZO = ZO; D.nc = NC; D.ncp = (NC + 3) / 4 * 4;
    D.NY = NY; D.NT = NT; D.MF = MF; D.NP = NP;
    D.n_teams = n_teams; D.team0 = 0;
    D.ysep = 1;              // a region of its own for the y results if LDS allows, else they overwrite u
    const int warm = c.hc.opt.warm_start ? 1 : 0;
    if (panel_lds_bytes(D, R, c.hc.opt.prec, warm) > 160 * 1024) D.ysep = 0;
    if (panel_lds_bytes(D, R, c.hc.opt.prec, warm) > 160 * 1024) return false;
    auto flat = [&](std::vector<int>& dst, size_t stride, int fill, auto get) {
        dst.assign((size_t)L * stride, fill);
        for (int l = 0; l < L; ++l) {
            const std::vector<int>& src = get(ws[l]);
            std::copy(src.begin(), src.end(), dst.begin() + (size_t)l * stride);
        }
    };
    auto flatd = [&](std::vector<double>& dst, size_t stride, auto get) {
        dst.assign((size_t)L * stride, 0.0);
        for (int l = 0; l < L; ++l) {
            const std::vector<double>& src = get(ws[l]);
            std::copy(src.begin(), src.end(), dst.begin() + (size_t)l * stride);
        }
    };
    c.tw_lo = P.leaf_lo; c.tw_nl = P.leaf_n;
    c.tw_nb.resize(L); c.pw_nx.resize(L); c.pw_ny.resize(L); c.pw_nt.resize(L); c.pw_np.resize(L);
    for (int l = 0; l < L; ++l) {
        c.tw_nb[l] = (int)ws[l].bglob.size();
        c.pw_nx[l] = (int)ws[l].fx.size();
        c.pw_ny[l] = (int)ws[l].yslot.size();
        c.pw_nt[l] = (int)ws[l].tk0.size();
        c.pw_np[l] = (int)ws[l].pubg.size();
    }
    flat(c.tozo, Hs, -1, [](W& w) -> std::vector<int>& { return w.ozo; });
    flat(c.topm, Hs, 0, [](W& w) -> std::vector<int>& { return w.opm; });
    flat(c.topc, Hs, 0, [](W& w) -> std::vector<int>& { return w.ops; });
    flat(c.topan, Hs, -1, [](W& w) -> std::vector<int>& { return w.opan; });
    flat(c.torp, NL + 1, 0, [](W& w) -> std::vector<int>& { return w.orp; });
    flat(c.tocol, NE, 0, [](W& w) -> std::vector<int>& { return w.ocol; });
    flat(c.tbglob, NB, 0, [](W& w) -> std::vector<int>& { return w.bglob; });
    flat(c.tbf, NB, 0, [](W& w) -> std::vector<int>& { return w.bf; });
    flat(c.tbt, NB, 0, [](W& w) -> std::vector<int>& { return w.bt; });
    flat(c.tbown, NB, 0, [](W& w) -> std::vector<int>& { return w.bown; });
    flat(c.tiptr, NL + 1, 0, [](W& w) -> std::vector<int>& { return w.iptr; });
    flat(c.tibr, NI, 0, [](W& w) -> std::vector<int>& { return w.ibrs; });
    flat(c.phbft, NB, 0, [](W& w) -> std::vector<int>& { return w.hbft; });
    flat(c.pxzsrc, XZ, 0, [](W& w) -> std::vector<int>& { return w.xzsrc; });
    flat(c.tsptr, NL + 1, 0, [](W& w) -> std::vector<int>& { return w.sptr; });
    flatd(c.toval, NE, [](W& w) -> std::vector<double>& { return w.oval; });
    flat(c.tosrc, NE, 0, [](W& w) -> std::vector<int>& { return w.osrc; });
    flatd(c.tbg, NB, [](W& w) -> std::vector<double>& { return w.bg; });
    flatd(c.tbal, NB, [](W& w) -> std::vector<double>& { return w.bal; });
    flatd(c.tsamp, NS, [](W& w) -> std::vector<double>& { return w.samp; });
    flatd(c.tsph, NS, [](W& w) -> std::vector<double>& { return w.sph; });
    flat(c.ppubr, NP, 0, [](W& w) -> std::vector<int>& { return w.pubr; });
    flat(c.ppubg, NP, 0, [](W& w) -> std::vector<int>& { return w.pubg; });
    flat(c.pxrow, NX, 0, [](W& w) -> std::vector<int>& { return w.fx; });
    flat(c.pxcol, NX, 0, [](W& w) -> std::vector<int>& { return w.xcol; });
    flat(c.pxzo, (size_t)NX * Hs, -1, [](W& w) -> std::vector<int>& { return w.xzo; });
    flat(c.pxpm, (size_t)NX * Hs, 0, [](W& w) -> std::vector<int>& { return w.xpm; });
    flat(c.pxps, (size_t)NX * Hs, 0, [](W& w) -> std::vector<int>& { return w.xps; });
    flat(c.pxpan, (size_t)NX * Hs, -1, [](W& w) -> std::vector<int>& { return w.xpan; });
    flat(c.pyslot, NY, -1, [](W& w) -> std::vector<int>& { return w.yslot; });
    flat(c.ptk0, NT, 0, [](W& w) -> std::vector<int>& { return w.tk0; });
    flat(c.ptnk, NT, 0, [](W& w) -> std::vector<int>& { return w.tnk; });
    flat(c.ptfo, NT, 0, [](W& w) -> std::vector<int>& { return w.tfo; });
    flat(c.pttile, NT, 0, [](W& w) -> std::vector<int>& { return w.ttile; });
    flat(c.pttp, NY / 16 + 1, 0, [](W& w) -> std::vector<int>& { return w.ttp; });
    flat(c.pttl, NT, 0, [](W& w) -> std::vector<int>& { return w.ttl; });
    flat(c.pwtask, kPanelWaves * kPanelYTasksPerWave, -1, [](W& w) -> std::vector<int>& { return w.wtask; });
    c.plpa = std::move(lpa);
    c.plpb = std::move(lpb);
    c.phlost = std::move(hlost);
    c.pw_xz.resize(L);
    for (int l = 0; l < L; ++l) c.pw_xz[l] = ws[l].xz;
    c.table_error = check_panel_tables(c, R);
    return c.table_error.empty();
}

// Workspace for the panel tables.
void carve_panel(emt_ctx& c, Arena& A)
{
    PanelDev& D = c.PD;
    const int64_t L = D.T, H = std::max(D.H, 1), TW = (int64_t)D.n_teams * D.T, R = c.R;
    auto ti = [&](int64_t cnt) { return A.take<int>(cnt); };
    auto td = [&](int64_t cnt) { return A.take<double>(cnt); };
    D.w_lo = ti(L); D.w_nl = ti(L); D.w_nb = ti(L); D.w_nx = ti(L); D.w_ny = ti(L); D.w_nt = ti(L);
    D.ozo = ti(L * H); D.opm = ti(L * H); D.ops = ti(L * H); D.opan = ti(L * H);
    D.orp = ti(L * (D.NL + 1)); D.ocol = ti(L * D.NE); D.oval = td(L * D.NE);
    D.bglob = ti(L * D.NB); D.bf = ti(L * D.NB); D.bt = ti(L * D.NB); D.bown = ti(L * D.NB);
    D.bg = td(L * D.NB); D.bal = td(L * D.NB);
    D.iptr = ti(L * (D.NL + 1)); D.ibr = ti(L * D.NI);
    D.sptr = ti(L * (D.NL + 1)); D.samp = td(L * D.NS); D.sph = td(L * D.NS);
    D.hbft = ti(L * D.NB); D.hlost = ti(TW * D.NB * kPanelCases);
    D.w_xz = ti(L); D.xzsrc = ti(L * D.XZ);
    D.w_np = ti(L); D.pubr = ti(L * D.NP); D.pubg = ti(L * D.NP);
    D.xrow = ti(L * D.NX); D.xcol = ti(L * D.NX);
    D.xzo = ti(L * D.NX * H); D.xpm = ti(L * D.NX * H); D.xps = ti(L * D.NX * H); D.xpan = ti(L * D.NX * H);
    D.yslot = ti(L * D.NY);
    D.tk0 = ti(L * D.NT); D.tnk = ti(L * D.NT); D.tfo = ti(L * D.NT); D.ttile = ti(L * D.NT);
    D.ttp = ti(L * (D.NY / 16 + 1)); D.ttl = ti(L * D.NT);
    D.wtask = ti(L * kPanelWaves * kPanelYTasksPerWave);
    D.mfr = td(L * D.MF);
    D.mfr32 = A.take<float>(L * D.MF);
    D.lpa = ti(TW * kPanelCases * R); D.lpb = ti(TW * kPanelCases * R);
    D.cpan = ti((int64_t)std::max(D.nc, 1) * H);
    D.am = td((int64_t)std::max(D.nc, 1) * std::max(D.nc, 1));
    D.bm = td((int64_t)std::max(D.nc, 1) * std::max(D.nc, 1));
    D.imgb = panel_image_bytes(D, (int)R, c.hc.opt.prec, c.hc.opt.warm_start ? 1 : 0);
    D.img = A.take<unsigned char>(L * (int64_t)D.imgb);
    D.sync = A.take<unsigned int>(TW);
    D.X0 = td((int64_t)D.n_teams * 2 * std::max(D.nc, 1) * kPanelCases);
    D.SP = td(TW * 2 * R * kPanelCases);
    D.VM = td(TW * 2 * kPanelCases);
}

// The panel's map y = M u and its A fragments, from the current FP64 hierarchy.
hinv_status build_panel_map(emt_ctx& c, hipStream_t s)
{
    PanelDev& D = c.PD;
    HIP_TRY(launch_coupling_map(c.hc.H, D.H, D.nc, D.cpan, D.am, D.bm, s));
    HIP_TRY(launch_panel_mfrag(D, s));
    HIP_TRY(launch_panel_image(D, c.E, c.hc.H, c.R, c.hc.opt.prec, c.hc.opt.warm_start ? 1 : 0, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HINV_OK;
}

hinv_status upload_panel(emt_ctx& c, hipStream_t s)
{
    PanelDev& D = c.PD;
    HIP_TRY(up(D.w_lo, c.tw_lo, s)); HIP_TRY(up(D.w_nl, c.tw_nl, s)); HIP_TRY(up(D.w_nb, c.tw_nb, s));
    HIP_TRY(up(D.w_nx, c.pw_nx, s)); HIP_TRY(up(D.w_ny, c.pw_ny, s)); HIP_TRY(up(D.w_nt, c.pw_nt, s));
    HIP_TRY(up(D.ozo, c.tozo, s)); HIP_TRY(up(D.opm, c.topm, s)); HIP_TRY(up(D.ops, c.topc, s));
    HIP_TRY(up(D.opan, c.topan, s));
    HIP_TRY(up(D.orp, c.torp, s)); HIP_TRY(up(D.ocol, c.tocol, s)); HIP_TRY(up(D.oval, c.toval, s));
    HIP_TRY(up(D.bglob, c.tbglob, s)); HIP_TRY(up(D.bf, c.tbf, s)); HIP_TRY(up(D.bt, c.tbt, s));
    HIP_TRY(up(D.bown, c.tbown, s)); HIP_TRY(up(D.bg, c.tbg, s)); HIP_TRY(up(D.bal, c.tbal, s));
    HIP_TRY(up(D.iptr, c.tiptr, s)); HIP_TRY(up(D.ibr, c.tibr, s)); HIP_TRY(up(D.sptr, c.tsptr, s));
    HIP_TRY(up(D.samp, c.tsamp, s)); HIP_TRY(up(D.sph, c.tsph, s));
    HIP_TRY(up(D.hbft, c.phbft, s)); HIP_TRY(up(D.hlost, c.phlost, s));
    HIP_TRY(up(D.w_xz, c.pw_xz, s)); HIP_TRY(up(D.xzsrc, c.pxzsrc, s));
    HIP_TRY(up(D.w_np, c.pw_np, s)); HIP_TRY(up(D.pubr, c.ppubr, s)); HIP_TRY(up(D.pubg, c.ppubg, s));
    HIP_TRY(up(D.xrow, c.pxrow, s)); HIP_TRY(up(D.xcol, c.pxcol, s));
    HIP_TRY(up(D.xzo, c.pxzo, s)); HIP_TRY(up(D.xpm, c.pxpm, s)); HIP_TRY(up(D.xps, c.pxps, s));
    HIP_TRY(up(D.xpan, c.pxpan, s));
    HIP_TRY(up(D.yslot, c.pyslot, s));
    HIP_TRY(up(D.tk0, c.ptk0, s)); HIP_TRY(up(D.tnk, c.ptnk, s)); HIP_TRY(up(D.tfo, c.ptfo, s));
    HIP_TRY(up(D.ttile, c.pttile, s)); HIP_TRY(up(D.ttp, c.pttp, s)); HIP_TRY(up(D.ttl, c.pttl, s));
    HIP_TRY(up(D.wtask, c.pwtask, s));
    HIP_TRY(up(D.lpa, c.plpa, s)); HIP_TRY(up(D.lpb, c.plpb, s));
    HIP_TRY(up(D.cpan, c.pcpan, s));
    HIP_TRY(hipMemsetAsync(D.sync, 0, (size_t)D.n_teams * D.T * sizeof(unsigned int), s));
    D.epoch0 = 0;
    HIP_TRY(panel_setup(D, c.R, c.hc.opt.prec, c.hc.opt.warm_start ? 1 : 0));
    HIP_TRY(hipStreamSynchronize(s));      // host tables may be rebuilt later
    return build_panel_map(c, s);
}

// ---------------------------------------------------------------------------
// Level plan (one case): per leaf its own rows, owned coupling columns per level with their
// S^{-1} rows, own Z panels, X rows (neighbours through G, then line-loss endpoints), CSR rows,
// branches and sources.  Per-leaf tables share the team layout's per-leaf vectors.
// Bounds check of the level engine's tables (see check_panel_tables).
std::string check_level_tables(const emt_ctx& c, int R)
{
    const Plan& P = c.hc.P;
    const LevelDev& D = c.LD;
    const int L = D.T, H = D.H, Hs = std::max(H, 1), n = c.n, nc = (int)P.col_row.size();
    char buf[256];
    auto bad = [&](const char* fmt, auto... a) {
        snprintf(buf, sizeof buf, fmt, a...);
        return std::string(buf);
    };
    auto mono = [&](const std::vector<int>& a, size_t at, int cnt, int cap) {
        if (a[at] != 0) return false;
        for (int i = 0; i < cnt; ++i)
            if (a[at + i + 1] < a[at + i]) return false;
        return a[at + cnt] <= cap;
    };
    for (int l = 0; l < L; ++l) {
        const int lo = c.tw_lo[l], nl = c.tw_nl[l], nx = c.lw_nx[l], nb = c.tw_nb[l];
        const int ncomb = nl + nx;
        if (lo < 0 || nl < 1 || nl > D.NL || lo + nl > n || nx < 0 || nx > D.NX || nb < 0 || nb > D.NB)
            return bad("leaf %d: counts out of range (lo %d nl %d nx %d nb %d)", l, lo, nl, nx, nb);
        for (int x = 0; x < nx; ++x) {
            const int r = c.lxrow[(size_t)l * D.NX + x];
            if (r < 0 || r >= n || (r >= lo && r < lo + nl)) return bad("leaf %d: X row %d (row %d) invalid", l, x, r);
        }
        for (int h = 0; h < H; ++h) {
            const size_t i = (size_t)l * Hs + h;
            const int zo = c.tozo[i], pm = c.topm[i], pc = c.topc[i];
            if (zo >= 0 && (pm < 1 || pm > D.PM || (int64_t)zo + (int64_t)pm * nl > D.ZO || pc < 0 || pc + pm > nc))
                return bad("leaf %d level %d: own Z rows (offset %d, %d columns from %d) out of bounds", l, h, zo, pm, pc);
        }
        if (!mono(c.loptr, (size_t)l * (H + 1), H, D.NO)) return bad("leaf %d: owned-column pointers invalid", l);
        for (int q = 0; q < c.loptr[(size_t)l * (H + 1) + H]; ++q) {
            const size_t i = (size_t)l * D.NO + q;
            const int g = c.locl[i], r = c.lorow[i], so = c.losoff[i];
            if (g < 0 || g >= nc || r < 0 || r >= nl || P.col_row[g] != lo + r || so < 0 ||
                so + P.node_m[P.col_node[g]] > D.SO)
                return bad("leaf %d: owned column %d (column %d, row %d, S^-1 offset %d) out of bounds", l, q, g, r, so);
        }
        const size_t rb = (size_t)l * (D.NL + 1);
        if (!mono(c.torp, rb, nl, D.NE) || !mono(c.tiptr, rb, nl, D.NI) || !mono(c.tsptr, rb, nl, D.NS))
            return bad("leaf %d: row pointers not monotone or beyond their tables", l);
        for (int e = 0; e < c.torp[rb + nl]; ++e)
            if (c.tocol[(size_t)l * D.NE + e] < 0 || c.tocol[(size_t)l * D.NE + e] >= ncomb)
                return bad("leaf %d: residual column %d out of range", l, c.tocol[(size_t)l * D.NE + e]);
        for (int e = 0; e < c.tiptr[rb + nl]; ++e)
            if (c.tibr[(size_t)l * D.NI + e] < 0 || c.tibr[(size_t)l * D.NI + e] >= nb)
                return bad("leaf %d: incident branch %d beyond %d branches", l, c.tibr[(size_t)l * D.NI + e], nb);
        for (int q = 0; q < nb; ++q) {
            const size_t i = (size_t)l * D.NB + q;
            if (c.tbglob[i] < 0 || c.tbglob[i] >= c.nbr || c.tbf[i] < 0 || c.tbf[i] >= ncomb || c.tbt[i] < 0 ||
                c.tbt[i] >= ncomb)
                return bad("leaf %d: branch %d (global %d, ends %d %d) out of range", l, q, c.tbglob[i], c.tbf[i], c.tbt[i]);
        }
        for (int j = 0; j < R; ++j) {
            const int a = c.llpa[(size_t)l * R + j], b = c.llpb[(size_t)l * R + j];
            if (a < -1 || a >= ncomb || b < -1 || b >= ncomb)
                return bad("leaf %d: change %d endpoint rows (%d, %d) out of range", l, j, a, b);
        }
    }
    return std::string();
}

bool build_level_plan(emt_ctx& c, int R)
{
    c.table_error.clear();
    const Plan& P = c.hc.P;
    const int L = (int)P.leaf_lo.size(), H = P.n_levels, NC = (int)P.col_row.size();
    if (c.n_cases != 1 || L < 1 || L > 256 || H < 0 || H > 7) return false;   // y tags hold the level in 3 bits
    std::vector<int> lpan((size_t)L * std::max(H, 1), -1);
    for (int l = 0; l < L; ++l) {
        for (int k = 0; k < P.anc_stride; ++k) {
            const int t = P.leaf_anc[(size_t)l * P.anc_stride + k];
            if (t < 0) break;
            const int h = P.node_level[t];
            for (int pp = P.node_pan0[t]; pp < P.node_pan0[t] + P.node_npan[t]; ++pp)
                if (P.pan_lo[pp] <= P.leaf_lo[l] && P.leaf_lo[l] < P.pan_lo[pp] + P.pan_n[pp]) lpan[(size_t)l * H + h - 1] = pp;
        }
    }
    std::vector<int> loss_rows;
    for (auto& x : c.losses[0]) {
        loss_rows.push_back(c.fr_p[x.second]);
        loss_rows.push_back(c.to_p[x.second]);
    }
    struct W {
        std::vector<int> xr, ozo, opm, opc, opan, optr, ocl, orow, osoff, orp, ocol, bglob, bf, bt, bown, iptr, ibr,
            sptr, lpa, lpb;
        std::vector<double> oval, bg, bal, samp, sph;
        std::vector<int> osrc;       // CSR entry of each oval value, plus one
        int zo = 0, so = 0;
    };
    std::vector<W> ws(L);
    int NL = 1, NX = 1, NB = 1, NE = 1, NI = 1, NS = 1, ZO = 1, NO = 1, SO = 1, PM = 1;
    for (size_t pp = 0; pp < P.pan_m.size(); ++pp) PM = std::max(PM, P.pan_m[pp]);
    for (int l = 0; l < L; ++l) {
        W& w = ws[l];
        const int lo = P.leaf_lo[l], nl = P.leaf_n[l];
        auto own = [&](int r) { return r >= lo && r < lo + nl; };
        for (int r = lo; r < lo + nl; ++r)
            for (int e = P.rp[r]; e < P.rp[r + 1]; ++e)
                if (!own(P.ci[e])) w.xr.push_back(P.ci[e]);
        std::sort(w.xr.begin(), w.xr.end());
        w.xr.erase(std::unique(w.xr.begin(), w.xr.end()), w.xr.end());
        for (int r : loss_rows)
            if (!own(r) && std::find(w.xr.begin(), w.xr.end(), r) == w.xr.end()) w.xr.push_back(r);
        auto comb = [&](int row) {
            return own(row) ? row - lo : nl + (int)(std::find(w.xr.begin(), w.xr.end(), row) - w.xr.begin());
        };
        // owned columns, grouped by level (columns are numbered level by level)
        w.optr.assign(H + 1, 0);
        for (int h = 1; h <= H; ++h) {
            for (int g = P.lvl_col[h - 1]; g < P.lvl_col[h]; ++g) {
                if (!own(P.col_row[g])) continue;
                w.ocl.push_back(g);
                w.orow.push_back(P.col_row[g] - lo);
                w.osoff.push_back(w.so);
                w.so += P.node_m[P.col_node[g]];
            }
            w.optr[h] = (int)w.ocl.size();
        }
        w.ozo.assign(H, -1); w.opm.assign(H, 0); w.opc.assign(H, 0); w.opan.assign(H, -1);
        for (int h = 1; h <= H; ++h) {
            const int pp = lpan[(size_t)l * H + h - 1];
            if (pp < 0) continue;
            w.opan[h - 1] = pp; w.ozo[h - 1] = w.zo; w.opm[h - 1] = P.pan_m[pp]; w.opc[h - 1] = P.pan_col0[pp];
            w.zo += P.pan_m[pp] * nl;
        }
        w.orp.assign(nl + 1, 0);
        for (int r = lo; r < lo + nl; ++r) {
            for (int e = P.rp[r]; e < P.rp[r + 1]; ++e) {
                w.ocol.push_back(comb(P.ci[e]));
                w.oval.push_back(P.cv[e]);
                w.osrc.push_back(e + 1);
            }
            w.orp[r - lo + 1] = (int)w.ocol.size();
        }
        std::vector<int> br;
        for (int r = lo; r < lo + nl; ++r)
            for (int q = c.inc_ptr[r]; q < c.inc_ptr[r + 1]; ++q) br.push_back(c.inc_br[q]);
        std::sort(br.begin(), br.end());
        br.erase(std::unique(br.begin(), br.end()), br.end());
        for (int e : br) {
            w.bglob.push_back(e);
            w.bf.push_back(comb(c.fr_p[e]));
            w.bt.push_back(comb(c.to_p[e]));
            w.bown.push_back(own(c.fr_p[e]) ? 1 : 0);
            w.bg.push_back(c.g[e]);
            w.bal.push_back(c.alpha[e]);
        }
        w.iptr.assign(nl + 1, 0);
        w.sptr.assign(nl + 1, 0);
        for (int r = lo; r < lo + nl; ++r) {
            for (int q = c.inc_ptr[r]; q < c.inc_ptr[r + 1]; ++q)
                w.ibr.push_back((int)(std::lower_bound(br.begin(), br.end(), c.inc_br[q]) - br.begin()));
            w.iptr[r - lo + 1] = (int)w.ibr.size();
            for (int q = c.src_ptr[r]; q < c.src_ptr[r + 1]; ++q) {
                w.samp.push_back(c.samp[q]);
                w.sph.push_back(c.sph[q]);
            }
            w.sptr[r - lo + 1] = (int)w.samp.size();
        }
        w.lpa.assign(R, -1);
        w.lpb.assign(R, -1);
        for (size_t j = 0; j < c.losses[0].size(); ++j) {
            w.lpa[j] = comb(c.fr_p[c.losses[0][j].second]);
            w.lpb[j] = comb(c.to_p[c.losses[0][j].second]);
        }
        NL = std::max(NL, nl); NX = std::max(NX, (int)w.xr.size()); NB = std::max(NB, (int)br.size());
        NE = std::max(NE, (int)w.ocol.size()); NI = std::max(NI, (int)w.ibr.size());
        NS = std::max(NS, (int)w.samp.size()); ZO = std::max(ZO, w.zo); NO = std::max(NO, (int)w.ocl.size());
        SO = std::max(SO, w.so);
    }
    (void)NC;
    if (c.level_nx_cap == 0) c.level_nx_cap = NX + 8;    // room for the endpoints of later line losses
    if (NX > c.level_nx_cap) return false;
    LevelDev& D = c.LD;
    D.T = L; D.H = H; D.NL = NL; D.NX = c.level_nx_cap; D.NB = NB; D.NE = NE; D.NI = NI; D.NS = NS; D.ZO = ZO;
    D.NO = NO; D.SO = SO; D.PM = PM;
    if (level_lds_bytes(D, R, c.hc.opt.prec, c.hc.opt.warm_start ? 1 : 0) > 160 * 1024) return false;
    const int Hs = std::max(H, 1);
    auto flat = [&](std::vector<int>& dst, size_t stride, auto get) {
        dst.assign((size_t)L * stride, 0);
        for (int l = 0; l < L; ++l) {
            const std::vector<int>& src = get(ws[l]);
            std::copy(src.begin(), src.end(), dst.begin() + (size_t)l * stride);
        }
    };
    auto flatd = [&](std::vector<double>& dst, size_t stride, auto get) {
        dst.assign((size_t)L * stride, 0.0);
        for (int l = 0; l < L; ++l) {
            const std::vector<double>& src = get(ws[l]);
            std::copy(src.begin(), src.end(), dst.begin() + (size_t)l * stride);
        }
    };
    c.tw_lo = P.leaf_lo; c.tw_nl = P.leaf_n;
    c.tw_nb.resize(L); c.lw_nx.resize(L);
    for (int l = 0; l < L; ++l) { c.tw_nb[l] = (int)ws[l].bglob.size(); c.lw_nx[l] = (int)ws[l].xr.size(); }
    flat(c.tozo, Hs, [](W& w) -> std::vector<int>& { return w.ozo; });
    flat(c.topm, Hs, [](W& w) -> std::vector<int>& { return w.opm; });
    flat(c.topc, Hs, [](W& w) -> std::vector<int>& { return w.opc; });
    flat(c.topan, Hs, [](W& w) -> std::vector<int>& { return w.opan; });
    flat(c.loptr, H + 1, [](W& w) -> std::vector<int>& { return w.optr; });
    flat(c.locl, NO, [](W& w) -> std::vector<int>& { return w.ocl; });
    flat(c.lorow, NO, [](W& w) -> std::vector<int>& { return w.orow; });
    flat(c.losoff, NO, [](W& w) -> std::vector<int>& { return w.osoff; });
    flat(c.lxrow, D.NX, [](W& w) -> std::vector<int>& { return w.xr; });
    flat(c.torp, NL + 1, [](W& w) -> std::vector<int>& { return w.orp; });
    flat(c.tocol, NE, [](W& w) -> std::vector<int>& { return w.ocol; });
    flat(c.tbglob, NB, [](W& w) -> std::vector<int>& { return w.bglob; });
    flat(c.tbf, NB, [](W& w) -> std::vector<int>& { return w.bf; });
    flat(c.tbt, NB, [](W& w) -> std::vector<int>& { return w.bt; });
    flat(c.tbown, NB, [](W& w) -> std::vector<int>& { return w.bown; });
    flat(c.tiptr, NL + 1, [](W& w) -> std::vector<int>& { return w.iptr; });
    flat(c.tibr, NI, [](W& w) -> std::vector<int>& { return w.ibr; });
    flat(c.tsptr, NL + 1, [](W& w) -> std::vector<int>& { return w.sptr; });
    flat(c.llpa, R, [](W& w) -> std::vector<int>& { return w.lpa; });
    flat(c.llpb, R, [](W& w) -> std::vector<int>& { return w.lpb; });
    flatd(c.toval, NE, [](W& w) -> std::vector<double>& { return w.oval; });
    flat(c.tosrc, NE, [](W& w) -> std::vector<int>& { return w.osrc; });
    flatd(c.tbg, NB, [](W& w) -> std::vector<double>& { return w.bg; });
    flatd(c.tbal, NB, [](W& w) -> std::vector<double>& { return w.bal; });
    flatd(c.tsamp, NS, [](W& w) -> std::vector<double>& { return w.samp; });
    flatd(c.tsph, NS, [](W& w) -> std::vector<double>& { return w.sph; });
    c.table_error = check_level_tables(c, R);
    return c.table_error.empty();
}

void carve_level(emt_ctx& c, Arena& A)
{
    LevelDev& D = c.LD;
    const int64_t L = D.T, Hs = std::max(D.H, 1), R = c.R;
    auto ti = [&](int64_t cnt) { return A.take<int>(cnt); };
    auto td = [&](int64_t cnt) { return A.take<double>(cnt); };
    D.w_lo = ti(L); D.w_nl = ti(L); D.w_nb = ti(L); D.w_nx = ti(L);
    D.ozo = ti(L * Hs); D.opm = ti(L * Hs); D.opc = ti(L * Hs); D.opan = ti(L * Hs);
    D.optr = ti(L * (D.H + 1)); D.ocl = ti(L * D.NO); D.orow = ti(L * D.NO); D.osoff = ti(L * D.NO);
    D.xrow = ti(L * D.NX);
    D.orp = ti(L * (D.NL + 1)); D.ocol = ti(L * D.NE); D.oval = td(L * D.NE);
    D.bglob = ti(L * D.NB); D.bf = ti(L * D.NB); D.bt = ti(L * D.NB); D.bown = ti(L * D.NB);
    D.bg = td(L * D.NB); D.bal = td(L * D.NB);
    D.iptr = ti(L * (D.NL + 1)); D.ibr = ti(L * D.NI);
    D.sptr = ti(L * (D.NL + 1)); D.samp = td(L * D.NS); D.sph = td(L * D.NS);
    D.lpa = ti(L * R); D.lpb = ti(L * R);
    D.sync = A.take<unsigned int>(L);
    D.Sx = td(2 * std::max<int64_t>((int64_t)c.hc.P.col_row.size(), 1));
    D.SL = A.take<unsigned long long>(2 * std::max<int64_t>((int64_t)c.hc.P.col_row.size(), 1));
    D.YL = A.take<unsigned long long>(2 * std::max<int64_t>((int64_t)c.hc.P.col_row.size(), 1));
    D.V1 = td(c.n);
    D.VL = A.take<unsigned long long>(2 * (int64_t)c.n);
    D.VM = td(L);
}

hinv_status upload_level(emt_ctx& c, hipStream_t s)
{
    LevelDev& D = c.LD;
    HIP_TRY(up(D.w_lo, c.tw_lo, s)); HIP_TRY(up(D.w_nl, c.tw_nl, s)); HIP_TRY(up(D.w_nb, c.tw_nb, s));
    HIP_TRY(up(D.w_nx, c.lw_nx, s));
    HIP_TRY(up(D.ozo, c.tozo, s)); HIP_TRY(up(D.opm, c.topm, s)); HIP_TRY(up(D.opc, c.topc, s));
    HIP_TRY(up(D.opan, c.topan, s));
    HIP_TRY(up(D.optr, c.loptr, s)); HIP_TRY(up(D.ocl, c.locl, s)); HIP_TRY(up(D.orow, c.lorow, s));
    HIP_TRY(up(D.osoff, c.losoff, s)); HIP_TRY(up(D.xrow, c.lxrow, s));
    HIP_TRY(up(D.orp, c.torp, s)); HIP_TRY(up(D.ocol, c.tocol, s)); HIP_TRY(up(D.oval, c.toval, s));
    HIP_TRY(up(D.bglob, c.tbglob, s)); HIP_TRY(up(D.bf, c.tbf, s)); HIP_TRY(up(D.bt, c.tbt, s));
    HIP_TRY(up(D.bown, c.tbown, s)); HIP_TRY(up(D.bg, c.tbg, s)); HIP_TRY(up(D.bal, c.tbal, s));
    HIP_TRY(up(D.iptr, c.tiptr, s)); HIP_TRY(up(D.ibr, c.tibr, s)); HIP_TRY(up(D.sptr, c.tsptr, s));
    HIP_TRY(up(D.samp, c.tsamp, s)); HIP_TRY(up(D.sph, c.tsph, s));
    HIP_TRY(up(D.lpa, c.llpa, s)); HIP_TRY(up(D.lpb, c.llpb, s));
    HIP_TRY(hipMemsetAsync(D.sync, 0, (size_t)D.T * sizeof(unsigned int), s));
    HIP_TRY(hipMemsetAsync(D.YL, 0, 2 * std::max<size_t>(c.hc.P.col_row.size(), 1) * sizeof(unsigned long long), s));   // tag 0: none
    HIP_TRY(hipMemsetAsync(D.VL, 0, 2 * (size_t)c.n * sizeof(unsigned long long), s));
    HIP_TRY(hipMemsetAsync(D.SL, 0, 2 * std::max<size_t>(c.hc.P.col_row.size(), 1) * sizeof(unsigned long long), s));
    HIP_TRY(hipStreamSynchronize(s));      // host tables may be rebuilt later
    return HINV_OK;
}

hinv_status upload_team(emt_ctx& c, hipStream_t s)
{
    TeamDev& D = c.TD;
    HIP_TRY(up(D.w_lo, c.tw_lo, s)); HIP_TRY(up(D.w_nl, c.tw_nl, s)); HIP_TRY(up(D.w_nx, c.tw_nx, s));
    HIP_TRY(up(D.w_nb, c.tw_nb, s)); HIP_TRY(up(D.w_nxu, c.tw_nxu, s)); HIP_TRY(up(D.xupd, c.txupd, s));
    HIP_TRY(up(D.uzo, c.tuzo, s));
    HIP_TRY(up(D.xrow, c.txrow, s)); HIP_TRY(up(D.xzo, c.txzo, s)); HIP_TRY(up(D.xpm, c.txpm, s));
    HIP_TRY(up(D.xpc, c.txpc, s)); HIP_TRY(up(D.xpan, c.txpan, s));
    HIP_TRY(up(D.ozo, c.tozo, s)); HIP_TRY(up(D.opm, c.topm, s)); HIP_TRY(up(D.opc, c.topc, s));
    HIP_TRY(up(D.opan, c.topan, s)); HIP_TRY(up(D.xpos, c.txpos, s));
    HIP_TRY(up(D.orp, c.torp, s)); HIP_TRY(up(D.ocol, c.tocol, s)); HIP_TRY(up(D.oval, c.toval, s));
    HIP_TRY(up(D.bglob, c.tbglob, s)); HIP_TRY(up(D.bf, c.tbf, s)); HIP_TRY(up(D.bt, c.tbt, s));
    HIP_TRY(up(D.bown, c.tbown, s)); HIP_TRY(up(D.bg, c.tbg, s)); HIP_TRY(up(D.bal, c.tbal, s));
    HIP_TRY(up(D.iptr, c.tiptr, s)); HIP_TRY(up(D.ibr, c.tibr, s)); HIP_TRY(up(D.sptr, c.tsptr, s));
    HIP_TRY(up(D.samp, c.tsamp, s)); HIP_TRY(up(D.sph, c.tsph, s)); HIP_TRY(up(D.csop, c.ttcso, s));
    HIP_TRY(up(D.cld, c.ttcld, s)); HIP_TRY(up(D.ylist, c.tylist, s)); HIP_TRY(up(D.w_ny, c.tw_ny, s));
    HIP_TRY(up(D.aoff, c.taoff, s)); HIP_TRY(up(D.alo, c.talo, s)); HIP_TRY(up(D.alen, c.talen, s));
    HIP_TRY(up(D.cpan, c.tcpan, s));
    HIP_TRY(hipMemsetAsync(D.sync, 0, (size_t)D.T * sizeof(unsigned int), s));
    HIP_TRY(launch_team_acoef(D, c.hc.H, s));
    HIP_TRY(hipStreamSynchronize(s));      // host tables may be rebuilt later
    return HINV_OK;
}

// Store the line changes of the given cases (from c.losses) in their change
// sets: u = G0^{-1} w for all of them in one batched FP64 apply, then the
// capacitance inverses.  Synchronises.
hinv_status load_case_losses(emt_ctx& c, const std::vector<int>& which, hipStream_t s)
{
    hinv_ctx& h = c.hc;
    const int n = c.n, R = c.R;
    std::vector<int> cols;    // (case*R + j) of each apply column
    std::vector<double> W;
    for (int k : which) {
        std::vector<int> a(R, -1), b(R, -1), act(R, INT32_MAX);
        std::vector<double> dg(R, 0.0);
        std::vector<int> lst(R, INT32_MAX), lbr(R, -1);
        const auto& L = c.losses[k];
        std::vector<double> d3, dinv3;
        if (c.ph == 3) {
            // a lost line is three changes, one per phase (w_p = e_from,p - e_to,p), coupled by
            // D = -Y of the line: G - W Y W^T removes the line's 3x3 companion; D^{-1} = -Z
            d3.assign(3 * (size_t)R, 0.0);
            dinv3.assign(3 * (size_t)R, 0.0);
            for (size_t j = 0; j < L.size(); ++j) {
                const int l = L[j].second;
                for (int p = 0; p < 3; ++p) {
                    const int i = 3 * (int)j + p, e = 3 * l + p;
                    a[i] = c.fr_p[e];
                    b[i] = c.to_p[e];
                    dg[i] = -c.y3[9 * l + 4 * p];
                    act[i] = lst[i] = L[j].first;
                    lbr[i] = e;
                    for (int q = 0; q < 3; ++q) {
                        d3[3 * i + q] = -c.y3[9 * l + 3 * p + q];
                        dinv3[3 * i + q] = -c.z3[9 * l + 3 * p + q];
                    }
                    cols.push_back(k * R + i);
                    std::vector<double> w(n, 0.0);
                    w[a[i]] = 1.0;
                    w[b[i]] = -1.0;
                    W.insert(W.end(), w.begin(), w.end());
                }
            }
            HIP_TRY(hipMemcpyAsync(c.m_d3 + (int64_t)k * R * 3, d3.data(), sizeof(double) * 3 * R,
                                   hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(c.m_dinv3 + (int64_t)k * R * 3, dinv3.data(), sizeof(double) * 3 * R,
                                   hipMemcpyHostToDevice, s));
        } else {
            for (size_t j = 0; j < L.size(); ++j) {
                const int e = L[j].second;
                a[j] = c.fr_p[e];
                b[j] = c.to_p[e];
                dg[j] = -c.g[e];
                act[j] = L[j].first;
                lst[j] = L[j].first;
                lbr[j] = e;
                cols.push_back(k * R + (int)j);
                std::vector<double> w(n, 0.0);
                w[a[j]] = 1.0;
                w[b[j]] = -1.0;
                W.insert(W.end(), w.begin(), w.end());
            }
        }
        const int cnt = c.ph * (int)L.size();
        HIP_TRY(hipMemcpyAsync((void*)(h.m_a + k * R), a.data(), sizeof(int) * R, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void*)(h.m_b + k * R), b.data(), sizeof(int) * R, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void*)(h.m_act + k * R), act.data(), sizeof(int) * R, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void*)(h.m_dg + k * R), dg.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void*)(h.m_count + k), &cnt, sizeof(int), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void*)(c.E.loss_step + k * R), lst.data(), sizeof(int) * R, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void*)(c.E.loss_br + k * R), lbr.data(), sizeof(int) * R, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync((void*)(c.E.loss_cnt + k), &cnt, sizeof(int), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));     // host vectors above are loop-local
    }
    // u = G0^{-1} w of every change, in groups of at most max_nrhs columns (the scratch X, Xo and Y hold
    // that many; a handle's changes can outnumber them once dynamic losses are added).  The apply treats
    // every column alone, so the grouping does not change any bit of u.
    const int nc = (int)cols.size();
    const int cap = std::max(1, h.opt.max_nrhs);
    for (int q0 = 0; q0 < nc; q0 += cap) {
        const int m = std::min(cap, nc - q0);
        HIP_TRY(hipMemcpyAsync(h.X, W.data() + (size_t)q0 * n, sizeof(double) * (size_t)m * n, hipMemcpyHostToDevice, s));
        launch_apply(h.H, h.P.lv.data(), HINV_FP64, h.X, h.Xo, h.Y, m, s);
        for (int q = 0; q < m; ++q) {
            double* dst = h.M.U + (int64_t)cols[q0 + q] * n;
            HIP_TRY(hipMemcpyAsync(dst, h.Xo + (int64_t)q * n, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            if (h.M.U32) launch_to_f32(dst, h.M.U32 + (int64_t)cols[q0 + q] * n, n, s);
        }
    }
    HIP_TRY(hipMemsetAsync(h.d_flags, 0, sizeof(int), s));
    launch_smw_capacitance(h.M, h.d_flags, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    int flags = 0;
    HIP_TRY(hipMemcpy(&flags, h.d_flags, sizeof(int), hipMemcpyDeviceToHost));
    if (flags & (kFlagNotSPD | kFlagSingular)) return fail(HINV_E_NOT_SPD, "a line loss makes G indefinite or singular");
    return HINV_OK;
}

// Rebuild the tables of the context's workgroup engine from the current
// plan: new line-loss endpoints must become exchange rows of every workgroup,
// and changed values of G must reach the rows kept for the residual.  Falls
// back to the hierarchical engines where a plan no longer fits.
hinv_status refresh_engine_tables(emt_ctx& c, hipStream_t s)
{
    hinv_status st = HINV_OK;
    if (c.engine == 3) {
        const bool ok = build_team_plan(c, c.R);
        if (!c.table_error.empty()) return fail(HINV_E_DEVICE, "team tables: %s", c.table_error.c_str());
        if (!ok) {
            c.engine = run_fits(c.hc.H) ? 2 : 1;
            c.team_ok = false;
        } else {
            st = upload_team(c, s);
        }
    } else if (c.engine == 5) {
        const bool ok = build_level_plan(c, c.R);
        if (!c.table_error.empty()) return fail(HINV_E_DEVICE, "level tables: %s", c.table_error.c_str());
        if (!ok) {
            c.engine = run_fits(c.hc.H) ? 2 : 1;
            c.level_ok = false;
        } else {
            st = upload_level(c, s);
        }
    } else if (c.engine == 4) {
        const bool ok = build_panel_plan(c, c.R);
        if (!c.table_error.empty()) return fail(HINV_E_DEVICE, "panel tables: %s", c.table_error.c_str());
        if (!ok) {
            c.engine = run_fits(c.hc.H) ? 2 : 1;
            c.panel_ok = false;
        } else {
            st = upload_panel(c, s);
        }
    }
    return st;
}

// After a change of values only (G's pattern kept), copy the new values of
// the given CSR entries into the workgroup engine's residual rows: a few
// element copies instead of a rebuild of every table.  Synchronises.
hinv_status patch_engine_values(emt_ctx& c, const std::vector<int>& entries, hipStream_t s)
{
    const double* d_oval = c.engine == 3 ? c.TD.oval : c.engine == 4 ? c.PD.oval : c.engine == 5 ? c.LD.oval : nullptr;
    if (!d_oval) return HINV_OK;
    const Plan& P = c.hc.P;
    for (size_t q = 0; q < c.tosrc.size(); ++q) {
        const int e = c.tosrc[q] - 1;
        if (e < 0 || std::find(entries.begin(), entries.end(), e) == entries.end()) continue;
        c.toval[q] = P.cv[e];
        HIP_TRY(hipMemcpyAsync((void*)(d_oval + q), &c.toval[q], sizeof(double), hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    return HINV_OK;
}

}  // namespace

extern "C" {

hinv_status emt_network_csr(const emt_network* net, int32_t* row_ptr, int32_t* col_idx, double* val, int64_t* nnz)
{
    if (!nnz) return fail(HINV_E_INVALID, "nnz is NULL");
    hinv_status st = check_network(net);
    if (st != HINV_OK) return st;
    std::vector<int> rp, ci;
    std::vector<double> cv;
    assemble_csr(net, rp, ci, cv);
    *nnz = (int64_t)ci.size();
    if (!row_ptr) return HINV_OK;
    if (!col_idx || !val) return fail(HINV_E_INVALID, "NULL output array");
    memcpy(row_ptr, rp.data(), sizeof(int) * rp.size());
    memcpy(col_idx, ci.data(), sizeof(int) * ci.size());
    memcpy(val, cv.data(), sizeof(double) * cv.size());
    return HINV_OK;
}

hinv_status emt_network3_csr(const emt_network* net, double mutual, int32_t* row_ptr, int32_t* col_idx, double* val,
                             int64_t* nnz)
{
    if (!nnz) return fail(HINV_E_INVALID, "nnz is NULL");
    hinv_status st = check_network(net);
    if (st != HINV_OK) return st;
    if (!(mutual >= 0.0 && mutual < 0.5)) return fail(HINV_E_INVALID, "mutual ratio %g outside [0, 0.5)", mutual);
    std::vector<int> rp, ci;
    std::vector<double> cv;
    assemble_csr3(net, mutual, rp, ci, cv);
    *nnz = (int64_t)ci.size();
    if (!row_ptr) return HINV_OK;
    if (!col_idx || !val) return fail(HINV_E_INVALID, "NULL output array");
    memcpy(row_ptr, rp.data(), sizeof(int) * rp.size());
    memcpy(col_idx, ci.data(), sizeof(int) * ci.size());
    memcpy(val, cv.data(), sizeof(double) * cv.size());
    return HINV_OK;
}

hinv_status emt_workspace_size(const emt_network* net, const hinv_tree* tree, const hinv_options* opt,
                               const emt_cases* cases, size_t* bytes)
{
    if (!bytes) return fail(HINV_E_INVALID, "bytes is NULL");
    std::unique_ptr<emt_ctx> c(new (std::nothrow) emt_ctx);
    if (!c) return fail(HINV_E_NO_MEMORY, "host allocation failed");
    std::vector<int> rp, ci;
    std::vector<double> cv;
    return emt_plan(net, tree, opt, cases, *c, rp, ci, cv, bytes);
}

// FNV-1a over the bytes of the caller's network (and three-phase parameters): a checkpoint resumes
// only on the network it was taken from.
static uint64_t network_hash(const emt_network* N, const Phase3* p3)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t bytes) {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t i = 0; i < bytes; ++i) h = (h ^ c[i]) * 1099511628211ull;
    };
    const int32_t ph = p3 ? 3 : 1;
    mix(&ph, sizeof ph);
    mix(&N->n_bus, sizeof N->n_bus);
    mix(&N->n_branch, sizeof N->n_branch);
    mix(&N->n_src, sizeof N->n_src);
    mix(&N->dt, sizeof N->dt);
    mix(&N->freq, sizeof N->freq);
    if (N->n_branch > 0) {
        mix(N->from, sizeof(int32_t) * N->n_branch);
        mix(N->to, sizeof(int32_t) * N->n_branch);
        mix(N->R, sizeof(double) * N->n_branch);
        mix(N->L, sizeof(double) * N->n_branch);
    }
    mix(N->C, sizeof(double) * N->n_bus);
    if (N->n_src > 0) {
        mix(N->src_bus, sizeof(int32_t) * N->n_src);
        mix(N->amp, sizeof(double) * N->n_src);
        mix(N->phase, sizeof(double) * N->n_src);
    }
    if (p3) {
        mix(&p3->mu, sizeof p3->mu);
        mix(p3->shift, sizeof p3->shift);
    }
    return h;
}

static hinv_status emt_create_impl(const emt_network* net, const Phase3* p3, const hinv_tree* tree,
                                   const hinv_options* opt, const emt_cases* cases, void* d_ws, size_t ws_bytes,
                                   void* stream, emt_handle* out)
{
    if (!out) return fail(HINV_E_INVALID, "out is NULL");
    *out = nullptr;
    std::unique_ptr<emt_ctx> c(new (std::nothrow) emt_ctx);
    if (!c) return fail(HINV_E_NO_MEMORY, "host allocation failed");
    std::vector<int> rp, ci;
    std::vector<double> cv;
    size_t need = 0;
    hinv_status st = emt_plan(net, tree, opt, cases, *c, rp, ci, cv, &need, p3);
    if (st != HINV_OK) return st;
    if (!d_ws) return fail(HINV_E_INVALID, "workspace is NULL");
    if (ws_bytes < need) return fail(HINV_E_NO_MEMORY, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    Arena A;
    A.base = (char*)d_ws;
    carve_hier(c->hc, A, c->n_cases, c->R, c->hc.opt.max_nrhs);
    carve_emt(*c, A, c->ph * net->n_src);
    if (c->team_ok) carve_team(*c, A);
    if (c->panel_ok) carve_panel(*c, A);
    if (c->level_ok) carve_level(*c, A);
    if (A.off > ws_bytes) return fail(HINV_E_NO_MEMORY, "workspace layout exceeds %zu bytes", ws_bytes);
    c->hc.M.R = c->R;
    EmtDev& E = c->E;
    E.dt = net->dt;
    E.omega = 2.0 * M_PI * net->freq;
    E.perm = c->hc.d_perm;
    HIP_TRY(up(E.fr, c->fr_p, s)); HIP_TRY(up(E.to, c->to_p, s)); HIP_TRY(up(E.g, c->g, s));
    HIP_TRY(up(E.alpha, c->alpha, s)); HIP_TRY(up(E.gC, c->gC, s));
    HIP_TRY(up(E.inc_ptr, c->inc_ptr, s)); HIP_TRY(up(E.inc_br, c->inc_br, s));
    HIP_TRY(up(E.src_ptr, c->src_ptr, s)); HIP_TRY(up(E.src_amp, c->samp, s)); HIP_TRY(up(E.src_ph, c->sph, s));
    if (c->ph == 3) {
        HIP_TRY(up(E.Y3, c->y3, s));
        HIP_TRY(up(E.A3, c->a3, s));
    }
    st = build_device(c->hc, s);        // synchronises
    if (st != HINV_OK) return st;
    if (c->team_ok) {
        st = upload_team(*c, s);
        if (st != HINV_OK) return st;
    }
    if (c->panel_ok) {
        st = upload_panel(*c, s);
        if (st != HINV_OK) return st;
    }
    if (c->level_ok) {
        st = upload_level(*c, s);
        if (st != HINV_OK) return st;
    }
    if (st != HINV_OK) return st;
    std::vector<int> all(c->n_cases);
    for (int k = 0; k < c->n_cases; ++k) all[k] = k;
    st = load_case_losses(*c, all, s);
    if (st != HINV_OK) return st;
    launch_emt_init(E, s);
    launch_set_rec(c->d_rec, RecParams{nullptr, nullptr, 0, 0}, s);
    HIP_TRY(hipMemsetAsync(c->d_applies, 0, sizeof(unsigned long long) * c->n_cases, s));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    c->step = 1;
    c->net_hash = network_hash(net, p3);
    *out = c.release();
    return HINV_OK;
}

hinv_status emt_create(const emt_network* net, const hinv_tree* tree, const hinv_options* opt,
                       const emt_cases* cases, void* d_ws, size_t ws_bytes, void* stream, emt_handle* out)
{
    return emt_create_impl(net, nullptr, tree, opt, cases, d_ws, ws_bytes, stream, out);
}

static Phase3 phase3_of(double mutual, const double* shift)
{
    Phase3 p3{mutual, {0.0, -2.0 * M_PI / 3.0, 2.0 * M_PI / 3.0}};
    if (shift)
        for (int p = 0; p < 3; ++p) p3.shift[p] = shift[p];
    return p3;
}

hinv_status emt3_workspace_size(const emt_network* net, double mutual, const double* shift, const hinv_tree* tree,
                                const hinv_options* opt, const emt_cases* cases, size_t* bytes)
{
    if (!bytes) return fail(HINV_E_INVALID, "bytes is NULL");
    std::unique_ptr<emt_ctx> c(new (std::nothrow) emt_ctx);
    if (!c) return fail(HINV_E_NO_MEMORY, "host allocation failed");
    std::vector<int> rp, ci;
    std::vector<double> cv;
    const Phase3 p3 = phase3_of(mutual, shift);
    return emt_plan(net, tree, opt, cases, *c, rp, ci, cv, bytes, &p3);
}

hinv_status emt3_create(const emt_network* net, double mutual, const double* shift, const hinv_tree* tree,
                        const hinv_options* opt, const emt_cases* cases, void* d_ws, size_t ws_bytes, void* stream,
                        emt_handle* out)
{
    const Phase3 p3 = phase3_of(mutual, shift);
    return emt_create_impl(net, &p3, tree, opt, cases, d_ws, ws_bytes, stream, out);
}

hinv_status emt_step(emt_handle h, int32_t n_steps, double* d_v_record, double* d_b_record, void* stream)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    if (n_steps < 0) return fail(HINV_E_INVALID, "n_steps < 0");
    if (n_steps == 0) return HINV_OK;
    emt_ctx& c = *h;
    hipStream_t s = (hipStream_t)stream;
    if (c.engine != 1) {
        RunParams P{c.step, n_steps, c.hc.opt.max_refine, c.hc.opt.rel_tol, c.hc.opt.warm_start ? 1 : 0,
                    d_v_record, d_b_record, c.hc.d_flags, c.hc.stats, c.d_applies, c.d_clock, c.clock_cap,
                    c.step, n_steps};
        if (c.engine == 3)
            HIP_TRY(launch_emt_team(c.TD, c.E, c.hc.H, c.hc.M, P, c.hc.opt.prec, s));
        else if (c.engine == 4) {
            // barrier epochs continue from the previous launch (the flags are never reset in between)
            const unsigned int per_step = c.hc.opt.prec == HINV_FP64 ? 1u : 1u + (unsigned)c.hc.opt.max_refine;
            if ((uint64_t)c.PD.epoch0 + (uint64_t)n_steps * per_step >= (1ull << 31)) {
                HIP_TRY(hipMemsetAsync(c.PD.sync, 0, (size_t)c.PD.n_teams * c.PD.T * sizeof(unsigned int), s));
                c.PD.epoch0 = 0;
            }
            HIP_TRY(launch_emt_panel(c.PD, c.E, c.hc.H, c.hc.M, P, c.hc.opt.prec, s));
            c.PD.epoch0 += (unsigned int)n_steps * per_step;
        }
        else if (c.engine == 5)
            HIP_TRY(launch_emt_level(c.LD, c.E, c.hc.H, c.hc.M, P, c.hc.opt.prec, s));
        else
            HIP_TRY(launch_emt_run(c.E, c.hc.H, c.hc.M, P, c.hc.opt.prec, s));
        c.step += n_steps;
        return HINV_OK;
    }
    launch_set_rec(c.d_rec, RecParams{d_v_record, d_b_record, c.step, n_steps}, s);
    // warm_start: every step starts from the previous step's v (FP64: the incremental form)
    const bool warm = c.hc.opt.warm_start && c.hc.opt.coupling == HINV_COUPLING_EXACT;
    for (int i = 0; i < n_steps; ++i) {
        if (warm)
            solve_from_previous(c.hc, c.E.b, c.E.v, c.n_cases, 1, c.E.step, s);
        else
            solve_new_order(c.hc, c.E.b, c.E.v, c.n_cases, 1, c.E.step, s);
        if (c.ph == 3)
            launch_emt_history3(c.E, c.d_rec, s);
        else
            launch_emt_history(c.E, c.d_rec, s);
    }
    HIP_TRY(hipGetLastError());
    c.step += n_steps;
    return HINV_OK;
}

hinv_status emt_lose_line(emt_handle h, int32_t case_idx, int32_t branch, void* stream)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    emt_ctx& c = *h;
    if (case_idx < 0 || case_idx >= c.n_cases) return fail(HINV_E_INVALID, "case %d out of range", case_idx);
    if (branch < 0 || branch >= c.nbr / c.ph) return fail(HINV_E_INVALID, "branch %d out of range", branch);
    auto& L = c.losses[case_idx];
    for (auto& x : L)
        if (x.second == branch) return fail(HINV_E_NO_SUCH_LINE, "branch %d is already lost in case %d", branch, case_idx);
    if (c.ph * ((int)L.size() + 1) > c.hc.opt.max_mod_rank)
        return fail(HINV_E_RANK_LIMIT, "case %d already has %d losses", case_idx, (int)L.size());
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    L.push_back({(int)c.step, branch});
    std::stable_sort(L.begin(), L.end());
    hinv_status st = load_case_losses(c, std::vector<int>{case_idx}, s);
    if (st != HINV_OK) {
        for (size_t j = 0; j < L.size(); ++j)
            if (L[j].second == branch) { L.erase(L.begin() + j); break; }
        load_case_losses(c, std::vector<int>{case_idx}, s);
        return st;
    }
    // b of the next step was assembled with the branch still in service
    launch_emt_rebuild_rhs(c.E, case_idx, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return refresh_engine_tables(c, s);
}

hinv_status emt_update_line(emt_handle h, int32_t a, int32_t b, double delta_g, void* stream,
                            hinv_update_info* out)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    emt_ctx& c = *h;
    if (c.ph == 3) return fail(HINV_E_INVALID, "emt_update_line takes single-phase networks only");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    LineEdit ed;
    hinv_status st = edit_line(c.hc, a, b, delta_g, s, ed);
    if (st != HINV_OK) return st;
    // every case's stored line losses were applied to the old inverse
    std::vector<int> all(c.n_cases);
    for (int k = 0; k < c.n_cases; ++k) all[k] = k;
    st = load_case_losses(c, all, s);
    if (st != HINV_OK) {
        const std::string why = g_err;
        hinv_status u = undo_line(c.hc, ed, s);
        if (u != HINV_OK) return u;
        u = load_case_losses(c, all, s);
        if (u != HINV_OK) return u;
        return fail(st, "%s (with the change of G between buses %d and %d)", why.c_str(), a, b);
    }
    std::vector<int> changed{ed.e_aa};
    for (int x : {ed.e_bb, ed.e_ab, ed.e_ba})
        if (x >= 0) changed.push_back(x);
    st = patch_engine_values(c, changed, s);
    if (st != HINV_OK) return st;
    if (c.engine == 3) {       // the rows a_g fold in S^{-1} and Z, which the rebuild changed
        HIP_TRY(launch_team_acoef(c.TD, c.hc.H, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (c.engine == 4) {       // so does the panel's map y = M u
        st = build_panel_map(c, s);
        if (st != HINV_OK) return st;
    }
    c.base_log.push_back({a, b, delta_g});
    if (out) fill_update_info(c.hc.P, ed.U, out);
    return HINV_OK;
}

// ---- checkpoints: header, base-matrix change log, per-case line losses, then the state vectors of
// every case in the caller's row and branch order (b, v, hC: rows; h: branches)
namespace {
struct StateHeader {
    char magic[8];
    uint32_t version;
    int32_t ph, n, nbr, n_cases, n_base, loss_slots, pad;
    int64_t step;
    uint64_t net_hash;
};
struct StateLoss {
    int32_t step, branch;
};
constexpr char kStateMagic[8] = {'H', 'I', 'N', 'V', 'E', 'M', 'T', 0};
constexpr uint32_t kStateVersion = 1;

size_t state_bytes(int n_base, int n_cases, int loss_slots, int n, int nbr)
{
    return sizeof(StateHeader) + sizeof(emt_ctx::BaseChange) * (size_t)n_base +
           (sizeof(int32_t) + sizeof(StateLoss) * (size_t)loss_slots) * (size_t)n_cases +
           sizeof(double) * (size_t)n_cases * (3 * (size_t)n + (size_t)nbr);
}
}  // namespace

hinv_status emt_state_size(emt_handle h, size_t* bytes)
{
    if (!h || !bytes) return fail(HINV_E_INVALID, "handle or bytes is NULL");
    const emt_ctx& c = *h;
    *bytes = state_bytes((int)c.base_log.size(), c.n_cases, c.R / c.ph, c.n, c.nbr);
    return HINV_OK;
}

hinv_status emt_save_state(emt_handle h, void* buf, size_t bytes, void* stream)
{
    if (!h || !buf) return fail(HINV_E_INVALID, "handle or buffer is NULL");
    emt_ctx& c = *h;
    const int slots = c.R / c.ph;
    const size_t need = state_bytes((int)c.base_log.size(), c.n_cases, slots, c.n, c.nbr);
    if (bytes < need) return fail(HINV_E_INVALID, "state buffer has %zu bytes, needs %zu", bytes, need);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    const int64_t K = c.n_cases, n = c.n, nbr = c.nbr;
    std::vector<double> dev((size_t)K * (3 * n + nbr));
    double* db = dev.data();
    double* dv = db + K * n;
    double* dh = dv + K * n;
    double* dhb = dh + K * n;
    HIP_TRY(hipMemcpy(db, c.E.b, sizeof(double) * K * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(dv, c.E.v, sizeof(double) * K * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(dh, c.E.hC, sizeof(double) * K * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(dhb, c.E.h + (c.step & 1) * K * nbr, sizeof(double) * K * nbr, hipMemcpyDeviceToHost));
    unsigned char* o = (unsigned char*)buf;
    StateHeader hd{};
    std::memcpy(hd.magic, kStateMagic, sizeof hd.magic);
    hd.version = kStateVersion;
    hd.ph = c.ph; hd.n = c.n; hd.nbr = c.nbr; hd.n_cases = c.n_cases;
    hd.n_base = (int32_t)c.base_log.size(); hd.loss_slots = slots;
    hd.step = c.step;
    hd.net_hash = c.net_hash;
    std::memcpy(o, &hd, sizeof hd);
    o += sizeof hd;
    if (!c.base_log.empty()) {
        std::memcpy(o, c.base_log.data(), sizeof(emt_ctx::BaseChange) * c.base_log.size());
        o += sizeof(emt_ctx::BaseChange) * c.base_log.size();
    }
    for (int k = 0; k < c.n_cases; ++k) {
        const int32_t cnt = (int32_t)c.losses[k].size();
        std::memcpy(o, &cnt, sizeof cnt);
        o += sizeof cnt;
        for (int j = 0; j < slots; ++j) {
            StateLoss L{0, -1};
            if (j < cnt) L = StateLoss{c.losses[k][j].first, c.losses[k][j].second};
            std::memcpy(o, &L, sizeof L);
            o += sizeof L;
        }
    }
    // rows to the caller's order (row r of the context is caller row perm[r])
    const std::vector<int>& perm = c.hc.P.perm;
    std::vector<double> rows((size_t)K * n);
    for (double* src : {db, dv, dh}) {
        for (int64_t k = 0; k < K; ++k)
            for (int64_t r = 0; r < n; ++r) rows[k * n + perm[r]] = src[k * n + r];
        std::memcpy(o, rows.data(), sizeof(double) * rows.size());
        o += sizeof(double) * rows.size();
    }
    std::memcpy(o, dhb, sizeof(double) * K * nbr);
    return HINV_OK;
}

hinv_status emt_load_state(emt_handle h, const void* buf, size_t bytes, void* stream)
{
    if (!h || !buf) return fail(HINV_E_INVALID, "handle or buffer is NULL");
    emt_ctx& c = *h;
    if (bytes < sizeof(StateHeader)) return fail(HINV_E_INVALID, "state buffer is shorter than its header");
    const unsigned char* o = (const unsigned char*)buf;
    StateHeader hd;
    std::memcpy(&hd, o, sizeof hd);
    o += sizeof hd;
    if (std::memcmp(hd.magic, kStateMagic, sizeof hd.magic) != 0 || hd.version != kStateVersion)
        return fail(HINV_E_INVALID, "not an EMT state of this library (magic or version)");
    if (hd.ph != c.ph || hd.n != c.n || hd.nbr != c.nbr || hd.n_cases != c.n_cases)
        return fail(HINV_E_INVALID, "state of %d cases x %d rows / %d branches (%d-phase); the handle has %d x %d / %d "
                    "(%d-phase)", hd.n_cases, hd.n, hd.nbr, hd.ph, c.n_cases, c.n, c.nbr, c.ph);
    if (hd.net_hash != c.net_hash) return fail(HINV_E_INVALID, "the state was taken on another network");
    if (hd.n_base < 0 || hd.loss_slots < 0 || hd.step < 1 || hd.step >= INT32_MAX)
        return fail(HINV_E_INVALID, "corrupt state header");
    const size_t need = state_bytes(hd.n_base, hd.n_cases, hd.loss_slots, hd.n, hd.nbr);
    if (bytes < need) return fail(HINV_E_INVALID, "state buffer has %zu bytes, its header needs %zu", bytes, need);
    std::vector<emt_ctx::BaseChange> log((size_t)hd.n_base);
    if (hd.n_base > 0) std::memcpy(log.data(), o, sizeof(emt_ctx::BaseChange) * log.size());
    o += sizeof(emt_ctx::BaseChange) * log.size();
    // the handle's own base-matrix changes must be where the state's began
    if (c.base_log.size() > log.size()) return fail(HINV_E_INVALID, "the handle has more base-matrix changes than the state");
    for (size_t i = 0; i < c.base_log.size(); ++i)
        if (c.base_log[i].a != log[i].a || c.base_log[i].b != log[i].b || c.base_log[i].dg != log[i].dg)
            return fail(HINV_E_INVALID, "base-matrix change %zu of the handle differs from the state's", i);
    std::vector<std::vector<std::pair<int, int>>> losses((size_t)c.n_cases);
    const int nlines = c.nbr / c.ph;
    for (int k = 0; k < c.n_cases; ++k) {
        int32_t cnt;
        std::memcpy(&cnt, o, sizeof cnt);
        o += sizeof cnt;
        if (cnt < 0 || cnt > hd.loss_slots || c.ph * cnt > c.hc.opt.max_mod_rank)
            return fail(HINV_E_RANK_LIMIT, "case %d of the state has %d line losses; the handle holds %d", k, cnt,
                        c.hc.opt.max_mod_rank / c.ph);
        for (int j = 0; j < hd.loss_slots; ++j) {
            StateLoss L;
            std::memcpy(&L, o, sizeof L);
            o += sizeof L;
            if (j >= cnt) continue;
            if (L.step < 1 || L.branch < 0 || L.branch >= nlines)
                return fail(HINV_E_INVALID, "case %d of the state has a bad loss (%d, %d)", k, L.step, L.branch);
            for (auto& x : losses[k])
                if (x.second == L.branch) return fail(HINV_E_INVALID, "case %d of the state loses branch %d twice", k, L.branch);
            losses[k].push_back({L.step, L.branch});
        }
        std::stable_sort(losses[k].begin(), losses[k].end());
    }
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamSynchronize(s));
    for (size_t i = c.base_log.size(); i < log.size(); ++i) {
        hinv_status st = emt_update_line(h, log[i].a, log[i].b, log[i].dg, stream, nullptr);
        if (st != HINV_OK) return st;
    }
    c.losses = std::move(losses);
    std::vector<int> all(c.n_cases);
    for (int k = 0; k < c.n_cases; ++k) all[k] = k;
    hinv_status st = load_case_losses(c, all, s);
    if (st != HINV_OK) return st;
    st = refresh_engine_tables(c, s);
    if (st != HINV_OK) return st;
    const int64_t K = c.n_cases, n = c.n, nbr = c.nbr;
    const std::vector<int>& perm = c.hc.P.perm;
    std::vector<double> rows((size_t)K * n), mine((size_t)K * n);
    for (double* dst : {c.E.b, c.E.v, c.E.hC}) {
        std::memcpy(rows.data(), o, sizeof(double) * rows.size());
        o += sizeof(double) * rows.size();
        for (int64_t k = 0; k < K; ++k)
            for (int64_t r = 0; r < n; ++r) mine[k * n + r] = rows[k * n + perm[r]];
        HIP_TRY(hipMemcpy(dst, mine.data(), sizeof(double) * mine.size(), hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(c.E.h + (hd.step & 1) * K * nbr, o, sizeof(double) * K * nbr, hipMemcpyHostToDevice));
    const int64_t step = hd.step;
    const unsigned int zero = 0;
    HIP_TRY(hipMemcpy(c.E.step, &step, sizeof step, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c.E.done, &zero, sizeof zero, hipMemcpyHostToDevice));
    c.step = step;
    return HINV_OK;
}

hinv_status emt_sync_status(emt_handle h)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    int flags[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpy(flags, h->hc.d_flags, sizeof flags, hipMemcpyDeviceToHost));
    int zero[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpy(h->hc.d_flags, zero, sizeof zero, hipMemcpyHostToDevice));
    if (flags[0] & kFlagBarrier) {
        if (h->engine == 4 && h->panel_ok) {   // a team stopped early: start the next launch from fresh flags
            HIP_TRY(hipMemset(h->PD.sync, 0, (size_t)h->PD.n_teams * h->PD.T * sizeof(unsigned int)));
            h->PD.epoch0 = 0;
        }
        return fail(HINV_E_DEVICE, "an inter-workgroup barrier timed out");
    }
    if (flags[0] & kFlagTeamRow) return fail(HINV_E_DEVICE, "a line change endpoint has no row in a workgroup's tables");
    if (flags[0] & (kFlagNotSPD | kFlagNaN)) return fail(HINV_E_NOT_SPD, "non-finite or indefinite result");
    if (flags[0] & kFlagNoConv) return fail(HINV_E_NO_CONVERGENCE, "refinement did not reach rel_tol");
    return HINV_OK;
}

hinv_status emt_get_step(emt_handle h, int64_t* step)
{
    if (!h || !step) return fail(HINV_E_INVALID, "NULL argument");
    *step = h->step;
    return HINV_OK;
}

hinv_status emt_get_stats(emt_handle h, int64_t* applies, double* max_rel_update)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    if (applies) {
        std::vector<unsigned long long> ap(h->n_cases);
        HIP_TRY(hipMemcpy(ap.data(), h->d_applies, sizeof(unsigned long long) * h->n_cases, hipMemcpyDeviceToHost));
        int64_t tot = h->hc.applies;
        for (auto a : ap) tot += (int64_t)a;
        *applies = tot;
    }
    if (max_rel_update) {
        std::vector<unsigned long long> st(h->n_cases);
        HIP_TRY(hipMemcpy(st.data(), h->hc.stats, sizeof(unsigned long long) * h->n_cases, hipMemcpyDeviceToHost));
        double m = 0.0;
        for (auto u : st) {
            double d;
            memcpy(&d, &u, sizeof d);
            m = std::max(m, d);
        }
        *max_rel_update = m;
    }
    return HINV_OK;
}

hinv_status emt_set_step_clock(emt_handle h, int64_t* d_clock, int64_t capacity)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    if (d_clock && capacity < 1) return fail(HINV_E_INVALID, "capacity must be >= 1");
    h->d_clock = d_clock;
    h->clock_cap = d_clock ? capacity : 0;
    return HINV_OK;
}

hinv_status hinv_wall_clock_khz(int32_t device, int32_t* khz)
{
    if (!khz) return fail(HINV_E_INVALID, "khz is NULL");
    int v = 0;
    HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, device));
    *khz = v;
    return HINV_OK;
}

hinv_status emt_destroy(emt_handle h)
{
    delete h;
    return HINV_OK;
}

}  // extern "C"

// =============================== serving ====================================
// Attached cases: those that fit one workgroup's LDS are slots of the one-workgroup-per-case
// serve launch; larger ones with a level plan are teams of one level launch; the rest run in
// the serve launch with their vectors in global memory.
struct serve_ctx {
    hinv_options opt{};
    int max_slots = 0;
    ServeSlot* d_slots = nullptr;
    LevelCase* d_lcases = nullptr;
    std::vector<ServeSlot> slot;       // per attached case (in attach order)
    std::vector<int> level;            // 1: stepped by the level launch
    std::vector<emt_ctx*> owner;       // handle of each attached case
    std::vector<int> ids;              // stable id of each attached case
    int next_id = 0;
    // dense launch tables (rebuilt on attach / detach)
    std::vector<ServeSlot> table;
    std::vector<LevelCase> ltable;
    std::vector<int> lwg;
    std::vector<unsigned int*> lsync;
    LevelDev Ld{};
    int lR = 1;
};

namespace {
hinv_status serve_upload(serve_ctx& S, hipStream_t s)
{
    S.table.clear();
    S.ltable.clear();
    S.lwg.clear();
    S.lsync.clear();
    S.Ld = LevelDev{};
    S.lR = 1;
    int wg0 = 0;
    for (size_t i = 0; i < S.slot.size(); ++i) {
        if (!S.level[i]) {
            S.table.push_back(S.slot[i]);
            continue;
        }
        const emt_ctx& c = *S.owner[i];
        const ServeSlot& sl = S.slot[i];
        LevelCase lc{};
        lc.D = c.LD;
        lc.E = c.E;
        lc.H = c.hc.H;
        lc.M = c.hc.M;
        lc.P = RunParams{0, 0, sl.max_refine, sl.rel_tol, S.opt.warm_start ? 1 : 0, sl.v_rec, nullptr, sl.flags,
                         sl.stats, sl.applies, nullptr, 0, sl.rec_step0, sl.rec_cap};
        lc.wg0 = wg0;
        wg0 += c.LD.T;
        S.ltable.push_back(lc);
        S.lwg.push_back(c.LD.T);
        S.lsync.push_back(c.LD.sync);
        LevelDev& L = S.Ld;
        L.NL = std::max(L.NL, c.LD.NL); L.NX = std::max(L.NX, c.LD.NX); L.NB = std::max(L.NB, c.LD.NB);
        L.NE = std::max(L.NE, c.LD.NE); L.NI = std::max(L.NI, c.LD.NI); L.NS = std::max(L.NS, c.LD.NS);
        L.ZO = std::max(L.ZO, c.LD.ZO); L.NO = std::max(L.NO, c.LD.NO); L.SO = std::max(L.SO, c.LD.SO);
        L.PM = std::max(L.PM, c.LD.PM); L.H = std::max(L.H, c.LD.H);
        S.lR = std::max(S.lR, c.hc.M.R);
    }
    if (!S.table.empty())
        HIP_TRY(hipMemcpyAsync(S.d_slots, S.table.data(), sizeof(ServeSlot) * S.table.size(), hipMemcpyHostToDevice, s));
    if (!S.ltable.empty())
        HIP_TRY(hipMemcpyAsync(S.d_lcases, S.ltable.data(), sizeof(LevelCase) * S.ltable.size(), hipMemcpyHostToDevice,
                               s));
    HIP_TRY(hipStreamSynchronize(s));
    return HINV_OK;
}
}  // namespace

extern "C" {

hinv_status serve_workspace_size(int32_t max_slots, size_t* bytes)
{
    if (!bytes || max_slots < 1) return fail(HINV_E_INVALID, "max_slots must be >= 1");
    *bytes = (sizeof(ServeSlot) + sizeof(LevelCase)) * (size_t)max_slots + 2 * kAlign;
    return HINV_OK;
}

hinv_status serve_create(const hinv_options* opt, int32_t max_slots, void* d_ws, size_t ws_bytes, serve_handle* out)
{
    if (!out) return fail(HINV_E_INVALID, "out is NULL");
    *out = nullptr;
    hinv_status st = check_options(opt, 1);
    if (st != HINV_OK) return st;
    if (opt->coupling != HINV_COUPLING_EXACT) return fail(HINV_E_INVALID, "serving needs coupling = HINV_COUPLING_EXACT");
    size_t need = 0;
    st = serve_workspace_size(max_slots, &need);
    if (st != HINV_OK) return st;
    if (!d_ws || ws_bytes < need) return fail(HINV_E_NO_MEMORY, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    std::unique_ptr<serve_ctx> c(new (std::nothrow) serve_ctx);
    if (!c) return fail(HINV_E_NO_MEMORY, "host allocation failed");
    c->opt = *opt;
    c->max_slots = max_slots;
    Arena A;
    A.base = (char*)d_ws;
    c->d_slots = A.take<ServeSlot>(max_slots);
    c->d_lcases = A.take<LevelCase>(max_slots);
    *out = c.release();
    return HINV_OK;
}

hinv_status serve_attach(serve_handle h, emt_handle e, double* d_v_record, int64_t record_capacity, void* stream,
                         int32_t* slot_id)
{
    if (!h || !e || !slot_id) return fail(HINV_E_INVALID, "NULL argument");
    serve_ctx& S = *h;
    emt_ctx& c = *e;
    if ((int)S.slot.size() >= S.max_slots) return fail(HINV_E_NO_MEMORY, "all %d slots are in use", S.max_slots);
    if (c.n_cases != 1) return fail(HINV_E_INVALID, "a served handle holds exactly one case");
    if (c.ph != 1) return fail(HINV_E_INVALID, "the serving pool takes single-phase networks only");
    if (c.hc.opt.prec != S.opt.prec || (c.hc.opt.warm_start != 0) != (S.opt.warm_start != 0))
        return fail(HINV_E_INVALID, "the case's precision / warm start differ from the pool's");
    for (emt_ctx* o : S.owner)
        if (o == e) return fail(HINV_E_INVALID, "the case is already attached");
    if (d_v_record && record_capacity < 1) return fail(HINV_E_INVALID, "record capacity must be >= 1");
    ServeSlot sl{};
    sl.E = c.E;
    sl.H = c.hc.H;
    sl.M = c.hc.M;
    sl.k = 0;
    sl.gvec = run_fits(c.hc.H) ? 0 : 1;
    sl.gscr = c.gscr;
    sl.v_rec = d_v_record;
    sl.rec_step0 = c.step;
    sl.rec_cap = d_v_record ? record_capacity : 0;
    sl.max_refine = c.hc.opt.max_refine;
    sl.rel_tol = c.hc.opt.rel_tol;
    sl.flags = c.hc.d_flags;
    sl.stats = c.hc.stats;
    sl.applies = c.d_applies;
    S.slot.push_back(sl);
    S.level.push_back(sl.gvec && c.level_ok ? 1 : 0);
    S.owner.push_back(e);
    S.ids.push_back(S.next_id);
    *slot_id = S.next_id++;
    return serve_upload(S, (hipStream_t)stream);
}

hinv_status serve_detach(serve_handle h, int32_t slot_id, void* stream)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    serve_ctx& S = *h;
    for (size_t i = 0; i < S.ids.size(); ++i) {
        if (S.ids[i] != slot_id) continue;
        HIP_TRY(hipStreamSynchronize((hipStream_t)stream));     // no launch may still read the table
        S.slot.erase(S.slot.begin() + i);
        S.level.erase(S.level.begin() + i);
        S.owner.erase(S.owner.begin() + i);
        S.ids.erase(S.ids.begin() + i);
        return serve_upload(S, (hipStream_t)stream);
    }
    return fail(HINV_E_INVALID, "no slot %d", slot_id);
}

hinv_status serve_step(serve_handle h, int32_t n_steps, void* stream)
{
    if (!h) return fail(HINV_E_INVALID, "handle is NULL");
    serve_ctx& S = *h;
    if (n_steps < 0) return fail(HINV_E_INVALID, "n_steps < 0");
    if (n_steps == 0 || S.slot.empty()) return HINV_OK;
    if (!S.table.empty()) {
        size_t lds = 0;
        for (const ServeSlot& sl : S.table) lds = std::max(lds, serve_lds_bytes(sl.H, sl.gvec != 0));
        if (lds > 160 * 1024) return fail(HINV_E_INVALID, "a served case's coupling levels exceed LDS");
        HIP_TRY(launch_emt_serve(S.d_slots, (int)S.table.size(), n_steps, lds, S.opt.prec, S.opt.warm_start,
                                 (hipStream_t)stream));
    }
    if (!S.ltable.empty()) {
        if (level_lds_bytes(S.Ld, S.lR, S.opt.prec, S.opt.warm_start ? 1 : 0) > 160 * 1024)
            return fail(HINV_E_INVALID, "the served cases' level tables exceed LDS together");
        HIP_TRY(launch_emt_level_multi(S.Ld, S.lR, S.d_lcases, S.lwg.data(), S.lsync.data(), (int)S.ltable.size(),
                                       n_steps, S.opt.prec, S.opt.warm_start, (hipStream_t)stream));
    }
    for (emt_ctx* o : S.owner) o->step += n_steps;
    return HINV_OK;
}

hinv_status serve_active(serve_handle h, int32_t* n_active)
{
    if (!h || !n_active) return fail(HINV_E_INVALID, "NULL argument");
    *n_active = (int32_t)h->slot.size();
    return HINV_OK;
}

hinv_status serve_destroy(serve_handle h)
{
    delete h;
    return HINV_OK;
}

}  // extern "C"
