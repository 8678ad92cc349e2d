// Host-only driver of the C ABI for the sanitizer run (AddressSanitizer and UndefinedBehaviorSanitizer
// on the host code; no GPU call): network assembly, workspace sizing of every engine (which builds and
// bounds-checks the engine plans), and the argument-validation paths, on networks written by the test.
// Input file: int32 n_bus, n_branch, n_src, n_nodes; double dt, freq; int32 from[], to[]; double R[],
// L[], C[]; int32 src_bus[]; double amp[], phase[]; int32 parent[], bus_leaf[].
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hinv.h"

namespace {

int g_checks = 0;

void expect(bool ok, const char* what)
{
    ++g_checks;
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%s)\n", what, hinv_last_error());
        std::exit(1);
    }
}

template <typename T>
std::vector<T> take(FILE* f, size_t n)
{
    std::vector<T> v(n);
    if (n && std::fread(v.data(), sizeof(T), n, f) != n) {
        std::fprintf(stderr, "short input file\n");
        std::exit(2);
    }
    return v;
}

struct Net {
    int32_t nb, nbr, ns, nn;
    double dt, freq;
    std::vector<int32_t> fr, to, sb, parent, leaf;
    std::vector<double> R, L, C, amp, ph;
    emt_network s;
    hinv_tree t;
};

Net load(const char* path)
{
    FILE* f = std::fopen(path, "rb");
    if (!f) {
        std::fprintf(stderr, "cannot open %s\n", path);
        std::exit(2);
    }
    Net n;
    auto hdr = take<int32_t>(f, 4);
    n.nb = hdr[0]; n.nbr = hdr[1]; n.ns = hdr[2]; n.nn = hdr[3];
    auto d = take<double>(f, 2);
    n.dt = d[0]; n.freq = d[1];
    n.fr = take<int32_t>(f, n.nbr); n.to = take<int32_t>(f, n.nbr);
    n.R = take<double>(f, n.nbr); n.L = take<double>(f, n.nbr); n.C = take<double>(f, n.nb);
    n.sb = take<int32_t>(f, n.ns); n.amp = take<double>(f, n.ns); n.ph = take<double>(f, n.ns);
    n.parent = take<int32_t>(f, n.nn); n.leaf = take<int32_t>(f, n.nb);
    std::fclose(f);
    n.s = emt_network{n.nb, n.nbr, n.fr.data(), n.to.data(), n.R.data(), n.L.data(), n.C.data(), n.dt,
                      n.ns, n.sb.data(), n.amp.data(), n.ph.data(), n.freq};
    n.t = hinv_tree{n.nn, n.parent.data(), n.leaf.data()};
    return n;
}

hinv_options opts(int prec, int rank, int mode, int warm)
{
    hinv_options o;
    std::memset(&o, 0, sizeof o);
    o.prec = (hinv_precision)prec;
    o.rel_tol = 1e-9;
    o.max_refine = 2;
    o.max_mod_rank = rank;
    o.max_nrhs = 1;
    o.warm_start = warm;
    o.kernel_mode = mode;
    o.coupling = HINV_COUPLING_EXACT;
    return o;
}

void run(const Net& n, int n_cases)
{
    // G as CSR: size query, then the arrays
    int64_t nnz = 0;
    expect(emt_network_csr(&n.s, nullptr, nullptr, nullptr, &nnz) == HINV_OK && nnz > 0, "csr size");
    std::vector<int32_t> rp(n.nb + 1), ci(nnz);
    std::vector<double> cv(nnz);
    expect(emt_network_csr(&n.s, rp.data(), ci.data(), cv.data(), &nnz) == HINV_OK, "csr");
    hinv_csr G{n.nb, rp.data(), ci.data(), cv.data()};
    size_t bytes = 0;
    for (int prec = 0; prec < 4; ++prec)
        for (int cpl = 0; cpl < 2; ++cpl) {
            hinv_options o = opts(prec, 2, 0, 0);
            o.coupling = (hinv_coupling)cpl;
            o.max_nrhs = 4;
            const hinv_status st = hinv_workspace_size(&G, &n.t, &o, &bytes);
            expect(st == HINV_OK || st == HINV_E_INVALID, "hinv_workspace_size");
        }
    expect(chol_workspace_size(&G, &bytes) == HINV_OK, "chol_workspace_size");
    // cases: two losses in even cases, one in odd ones, spread over the branches
    std::vector<int32_t> ptr(n_cases + 1), st, br;
    for (int k = 0; k < n_cases; ++k) {
        ptr[k] = (int32_t)st.size();
        for (int j = 0; j < 2 - (k % 2); ++j) {
            st.push_back(10 + 7 * k + j);
            br.push_back((int32_t)((k * 37 + j * 11) % n.nbr));
        }
        ptr[k + 1] = (int32_t)st.size();
    }
    emt_cases cs{n_cases, ptr.data(), st.data(), br.data()};
    for (int mode = 0; mode <= 5; ++mode)
        for (int prec : {0, 1, 2})
            for (int warm : {0, 1}) {
                hinv_options o = opts(prec, 2, mode, warm);
                const hinv_status s = emt_workspace_size(&n.s, &n.t, &o, &cs, &bytes);
                expect(s == HINV_OK || s == HINV_E_INVALID, "emt_workspace_size");
            }
    std::vector<int32_t> rp3(3 * n.nb + 1);
    int64_t nnz3 = 0;
    expect(emt_network3_csr(&n.s, 0.3, nullptr, nullptr, nullptr, &nnz3) == HINV_OK, "csr3 size");
    std::vector<int32_t> ci3(nnz3);
    std::vector<double> cv3(nnz3);
    expect(emt_network3_csr(&n.s, 0.3, rp3.data(), ci3.data(), cv3.data(), &nnz3) == HINV_OK, "csr3");
    {
        hinv_options o = opts(0, 6, 0, 0);
        const hinv_status s = emt3_workspace_size(&n.s, 0.3, nullptr, &n.t, &o, &cs, &bytes);
        expect(s == HINV_OK || s == HINV_E_INVALID, "emt3_workspace_size");
    }
    expect(serve_workspace_size(64, &bytes) == HINV_OK, "serve_workspace_size");
    // validation paths: every one returns an error and leaves a message
    hinv_options o = opts(0, 2, 0, 0);
    expect(emt_workspace_size(nullptr, &n.t, &o, &cs, &bytes) == HINV_E_INVALID, "NULL network");
    expect(emt_workspace_size(&n.s, nullptr, &o, &cs, &bytes) == HINV_E_INVALID, "NULL tree");
    expect(emt_workspace_size(&n.s, &n.t, nullptr, &cs, &bytes) == HINV_E_INVALID, "NULL options");
    Net bad = n;
    bad.fr[0] = n.nb;                                   // a branch end outside the buses
    bad.s.from = bad.fr.data(); bad.s.to = bad.to.data(); bad.s.R = bad.R.data(); bad.s.L = bad.L.data();
    bad.s.C = bad.C.data(); bad.s.src_bus = bad.sb.data(); bad.s.amp = bad.amp.data(); bad.s.phase = bad.ph.data();
    expect(emt_workspace_size(&bad.s, &n.t, &o, &cs, &bytes) == HINV_E_INVALID, "bad branch");
    expect(emt_network_csr(&bad.s, nullptr, nullptr, nullptr, &nnz) == HINV_E_INVALID, "bad branch csr");
    std::vector<int32_t> br2 = br;
    br2[0] = n.nbr + 5;                                 // a loss of a branch that does not exist
    emt_cases cs2{n_cases, ptr.data(), st.data(), br2.data()};
    expect(emt_workspace_size(&n.s, &n.t, &o, &cs2, &bytes) == HINV_E_INVALID, "bad loss branch");
    hinv_options o1 = opts(0, 1, 0, 0);                 // case 0 has two losses: rank 1 cannot hold them
    expect(emt_workspace_size(&n.s, &n.t, &o1, &cs, &bytes) != HINV_OK, "rank limit");
    std::vector<int32_t> par = n.parent;
    par[0] = 0;                                         // a tree node that is its own parent
    hinv_tree t2{n.nn, par.data(), n.leaf.data()};
    expect(emt_workspace_size(&n.s, &t2, &o, &cs, &bytes) == HINV_E_INVALID, "cyclic tree");
    expect(hinv_workspace_size(&G, &n.t, nullptr, &bytes) == HINV_E_INVALID, "NULL options (hinv)");
    expect(std::strlen(hinv_last_error()) > 0, "last error message");
}

}  // namespace

int main(int argc, char** argv)
{
    for (int i = 1; i < argc; ++i) {
        const Net n = load(argv[i]);
        run(n, 1);
        run(n, 17);
        std::printf("%s: ok\n", argv[i]);
    }
    std::printf("sanitize driver: %d checks passed\n", g_checks);
    return 0;
}
