/*
 * FP64 CPU oracle for the EMT network solution — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct loops.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may call this code; the GPU library
 * never links it and shares no source with it.
 *
 * What it computes (paper, Section II, Eq. (1)-(2)): the nodal network
 * equation G v = i_in + i_his is solved exactly, either by LU factorisation
 * with partial pivoting (the "LU-based" solver the paper compares against) or
 * by multiplying with an explicit inverse G^{-1} obtained by solving G X = I.
 *
 * G comes from trapezoidal companion models (the paper's Section II only says
 * the network is discretised by numerical integration; the trapezoidal rule is
 * the standard EMTP choice): a series R-L branch becomes a conductance
 * g = 1 / (R + 2L/dt) between its buses, a shunt C a conductance 2C/dt to
 * ground.
 *
 * Matrices are dense, row-major, n x n.  OpenMP only splits independent rows
 * or columns; the arithmetic of each entry is the sequential definition.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Dense G of the network; branches with alive[e] == 0 are left out
 * (alive may be NULL: all branches present).  Returns 0, or -1 on a bad index. */
int orc_assemble(int n, int nbr, const int* fr, const int* to, const double* R, const double* L,
                 const double* C, double dt, const unsigned char* alive, double* G)
{
    memset(G, 0, sizeof(double) * (size_t)n * (size_t)n);
    for (int a = 0; a < n; ++a) G[(size_t)a * n + a] += 2.0 * C[a] / dt;
    for (int e = 0; e < nbr; ++e) {
        if (alive && !alive[e]) continue;
        int a = fr[e], b = to[e];
        if (a < 0 || a >= n || b < 0 || b >= n || a == b) return -1;
        double g = 1.0 / (R[e] + 2.0 * L[e] / dt);
        G[(size_t)a * n + a] += g;
        G[(size_t)b * n + b] += g;
        G[(size_t)a * n + b] -= g;
        G[(size_t)b * n + a] -= g;
    }
    return 0;
}

/* In-place LU with partial pivoting: P A = L U, L unit lower.  At step k row k
 * is swapped with row piv[k].  Returns 0, or -(k+1) if column k has no
 * non-zero pivot. */
int orc_lu_factor(int n, double* A, int* piv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(A[(size_t)i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (best == 0.0) return -(k + 1);
        if (p != k)
            for (int j = 0; j < n; ++j) {
                double t = A[(size_t)k * n + j];
                A[(size_t)k * n + j] = A[(size_t)p * n + j];
                A[(size_t)p * n + j] = t;
            }
        const double* rk = A + (size_t)k * n;
#pragma omp parallel for schedule(static) if (n - k > 256)
        for (int i = k + 1; i < n; ++i) {
            double* ri = A + (size_t)i * n;
            double l = ri[k] / rk[k];
            ri[k] = l;
            for (int j = k + 1; j < n; ++j) ri[j] -= l * rk[j];
        }
    }
    return 0;
}

/* Solve A x = b with the factors of orc_lu_factor; x holds b on entry. */
void orc_lu_solve(int n, const double* LU, const int* piv, double* x)
{
    for (int k = 0; k < n; ++k) {
        int p = piv[k];
        if (p != k) { double t = x[k]; x[k] = x[p]; x[p] = t; }
    }
    for (int i = 0; i < n; ++i) {
        double s = x[i];
        for (int j = 0; j < i; ++j) s -= LU[(size_t)i * n + j] * x[j];
        x[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int j = i + 1; j < n; ++j) s -= LU[(size_t)i * n + j] * x[j];
        x[i] = s / LU[(size_t)i * n + i];
    }
}

/* Solve G x = b (G unchanged).  Returns the factorisation status. */
int orc_solve(int n, const double* G, const double* b, double* x)
{
    double* A = (double*)malloc(sizeof(double) * (size_t)n * n);
    int* piv = (int*)malloc(sizeof(int) * (size_t)n);
    if (!A || !piv) { free(A); free(piv); return -1000000; }
    memcpy(A, G, sizeof(double) * (size_t)n * n);
    int st = orc_lu_factor(n, A, piv);
    if (st == 0) {
        memcpy(x, b, sizeof(double) * (size_t)n);
        orc_lu_solve(n, A, piv, x);
    }
    free(A);
    free(piv);
    return st;
}

/* Factor once and solve nrhs right-hand sides stored as rows of B (nrhs x n). */
int orc_solve_many(int n, const double* G, int nrhs, const double* B, double* X)
{
    double* A = (double*)malloc(sizeof(double) * (size_t)n * n);
    int* piv = (int*)malloc(sizeof(int) * (size_t)n);
    if (!A || !piv) { free(A); free(piv); return -1000000; }
    memcpy(A, G, sizeof(double) * (size_t)n * n);
    int st = orc_lu_factor(n, A, piv);
    if (st == 0) {
#pragma omp parallel for schedule(dynamic)
        for (int r = 0; r < nrhs; ++r) {
            memcpy(X + (size_t)r * n, B + (size_t)r * n, sizeof(double) * (size_t)n);
            orc_lu_solve(n, A, piv, X + (size_t)r * n);
        }
    }
    free(A);
    free(piv);
    return st;
}

/* Explicit inverse: column j of Ginv solves G x = e_j.  Row-major output. */
int orc_inverse(int n, const double* G, double* Ginv)
{
    double* A = (double*)malloc(sizeof(double) * (size_t)n * n);
    int* piv = (int*)malloc(sizeof(int) * (size_t)n);
    if (!A || !piv) { free(A); free(piv); return -1000000; }
    memcpy(A, G, sizeof(double) * (size_t)n * n);
    int st = orc_lu_factor(n, A, piv);
    if (st == 0) {
#pragma omp parallel
        {
            double* x = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(dynamic, 8)
            for (int j = 0; j < n; ++j) {
                for (int i = 0; i < n; ++i) x[i] = (i == j) ? 1.0 : 0.0;
                orc_lu_solve(n, A, piv, x);
                for (int i = 0; i < n; ++i) Ginv[(size_t)i * n + j] = x[i];
            }
            free(x);
        }
    }
    free(A);
    free(piv);
    return st;
}

/* y = M x for a dense row-major n x n matrix (the explicit-inverse solve). */
void orc_matvec(int n, const double* M, const double* x, double* y)
{
#pragma omp parallel for schedule(static) if (n > 512)
    for (int i = 0; i < n; ++i) {
        const double* r = M + (size_t)i * n;
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += r[j] * x[j];
        y[i] = s;
    }
}
