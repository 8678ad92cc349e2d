// EMT time stepping around the network solution (paper Section II, Eq. (1)):
// G v(t) = i_in(t) + i_his(t - dt), with trapezoidal companion models.
//
//   series R-L branch e (from f to t):  i_e^n = g v_ft^n + h_e^n,
//        h_e^{n+1} = g v_ft^n + alpha i_e^n,  g = 1/(R + 2L/dt), alpha = g (2L/dt - R)
//   shunt C at bus a:                    i_C^n = gC v_a^n + hC_a^n,
//        hC_a^{n+1} = -gC v_a^n - i_C^n,     gC = 2C/dt
//   right-hand side  b^{n+1}_a = i_in,a(t_{n+1}) - sum_e A[a,e] h_e^{n+1} - hC_a^{n+1}
//        with A[a,e] = +1 if a is the branch's from-bus, -1 if its to-bus.
// A branch lost at step s carries no current from step s on: its history is
// zero and it contributes nothing to b from step s on.
//
// One thread per (bus, case).  Each bus recomputes the new history of its
// incident branches itself (both endpoints compute the identical value; the
// from-bus stores it), so the pass needs no atomics and no second launch.
#include "hinv_internal.h"

namespace hinv {

__device__ inline bool lost_by(const EmtDev& E, int k, int e, int64_t step)
{
    const int cnt = E.loss_cnt[k];
    for (int j = 0; j < cnt; ++j)
        if (E.loss_br[k * E.R + j] == e && (int64_t)E.loss_step[k * E.R + j] <= step) return true;
    return false;
}

__device__ inline double source_at(const EmtDev& E, int a, double t)
{
    double s = 0.0;
    for (int q = E.src_ptr[a]; q < E.src_ptr[a + 1]; ++q) s += E.src_amp[q] * sin(E.omega * t + E.src_ph[q]);
    return s;
}

// Start: v = 0, branch currents 0, capacitor currents consistent with KCL at
// t = 0 (i_C(0) = i_in(0)), so hC^1 = -i_in(0) and b^1 = i_in(t_1) - hC^1.
__global__ __launch_bounds__(kBlock) void k_emt_init(EmtDev E)
{
    const int k = blockIdx.y;
    for (int a = blockIdx.x * kBlock + threadIdx.x; a < E.n; a += gridDim.x * kBlock) {
        const int64_t idx = (int64_t)k * E.n + a;
        const double hc = -source_at(E, a, 0.0);
        E.hC[idx] = hc;
        E.v[idx] = 0.0;
        E.b[idx] = source_at(E, a, 1.0 * E.dt) - hc;
    }
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < E.nbr; e += gridDim.x * kBlock) {
        E.h[(int64_t)k * E.nbr + e] = 0.0;
        E.h[(int64_t)E.n_cases * E.nbr + (int64_t)k * E.nbr + e] = 0.0;
    }
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        *E.step = 1;
        *E.done = 0;
    }
}

void launch_emt_init(const EmtDev& E, hipStream_t s)
{
    int gx = (E.n > E.nbr ? E.n : E.nbr);
    gx = (gx + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_emt_init, dim3(gx, E.n_cases), dim3(kBlock), 0, s, E);
}

__global__ __launch_bounds__(kBlock) void k_emt_history(EmtDev E, const RecParams* __restrict__ rec)
{
    const int k = blockIdx.y;
    const int a = blockIdx.x * kBlock + threadIdx.x;
    const int64_t step = *E.step;
    if (a < E.n) {
        const int64_t base = (int64_t)k * E.n;
        const double* v = E.v + base;
        const double* hcur = E.h + (int64_t)(step & 1) * E.n_cases * E.nbr + (int64_t)k * E.nbr;
        double* hnext = E.h + (int64_t)((step + 1) & 1) * E.n_cases * E.nbr + (int64_t)k * E.nbr;
        const double va = v[a];
        double bn = source_at(E, a, (double)(step + 1) * E.dt);
        for (int q = E.inc_ptr[a]; q < E.inc_ptr[a + 1]; ++q) {
            const int e = E.inc_br[q];
            const int f = E.fr[e], t = E.to[e];
            double hn = 0.0;
            if (!lost_by(E, k, e, step + 1)) {
                const double vft = v[f] - v[t];
                const double ie = E.g[e] * vft + hcur[e];
                hn = E.g[e] * vft + E.alpha[e] * ie;
            }
            bn -= (a == f) ? hn : -hn;
            if (a == f) hnext[e] = hn;
        }
        const double ic = E.gC[a] * va + E.hC[base + a];
        const double hcn = -E.gC[a] * va - ic;
        E.hC[base + a] = hcn;
        bn -= hcn;
        const int64_t j = step - rec->step0;
        if (j >= 0 && j < rec->nsteps) {
            const int64_t o = (j * E.n_cases + k) * (int64_t)E.n + E.perm[a];
            if (rec->v) rec->v[o] = va;
            if (rec->b) rec->b[o] = E.b[base + a];
        }
        E.b[base + a] = bn;
    }
    // the last block to finish advances the step counter
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int total = gridDim.x * gridDim.y;
        const unsigned int prev = atomicAdd(E.done, 1u);
        if (prev == total - 1) {
            *E.done = 0;
            __threadfence();
            *E.step = step + 1;
        }
    }
}

void launch_emt_history(const EmtDev& E, const RecParams* rec, hipStream_t s)
{
    hipLaunchKernelGGL(k_emt_history, dim3((E.n + kBlock - 1) / kBlock, E.n_cases), dim3(kBlock), 0, s, E, rec);
}

// Three-phase networks (rows are bus phases; branch 3l+p is phase p of line l).  Line l's companion is
// the 3x3 admittance Y = Y3[l] with history weight A = A3[l]:
//   i_l^n = Y v_ft^n + h_l^n,   h_l^{n+1} = Y v_ft^n + A i_l^n      (3-vectors, v_ft = v_from - v_to)
// so the new history of phase p needs the voltages and histories of all three phases of the line.
// Same threading as k_emt_history: one thread per (row, case); each row recomputes its incident
// phase-branches' histories in one fixed operation order, so both ends of a line agree bitwise.
__global__ __launch_bounds__(kBlock) void k_emt_history3(EmtDev E, const RecParams* __restrict__ rec)
{
    const int k = blockIdx.y;
    const int a = blockIdx.x * kBlock + threadIdx.x;
    const int64_t step = *E.step;
    if (a < E.n) {
        const int64_t base = (int64_t)k * E.n;
        const double* v = E.v + base;
        const double* hcur = E.h + (int64_t)(step & 1) * E.n_cases * E.nbr + (int64_t)k * E.nbr;
        double* hnext = E.h + (int64_t)((step + 1) & 1) * E.n_cases * E.nbr + (int64_t)k * E.nbr;
        const double va = v[a];
        double bn = source_at(E, a, (double)(step + 1) * E.dt);
        for (int q = E.inc_ptr[a]; q < E.inc_ptr[a + 1]; ++q) {
            const int e = E.inc_br[q];
            const int l = e / 3, p = e - 3 * l;
            double hn = 0.0;
            if (!lost_by(E, k, e, step + 1)) hn = line3_history(E, v, hcur, l, p);
            bn -= (a == E.fr[e]) ? hn : -hn;
            if (a == E.fr[e]) hnext[e] = hn;
        }
        const double ic = E.gC[a] * va + E.hC[base + a];
        const double hcn = -E.gC[a] * va - ic;
        E.hC[base + a] = hcn;
        bn -= hcn;
        const int64_t j = step - rec->step0;
        if (j >= 0 && j < rec->nsteps) {
            const int64_t o = (j * E.n_cases + k) * (int64_t)E.n + E.perm[a];
            if (rec->v) rec->v[o] = va;
            if (rec->b) rec->b[o] = E.b[base + a];
        }
        E.b[base + a] = bn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int total = gridDim.x * gridDim.y;
        const unsigned int prev = atomicAdd(E.done, 1u);
        if (prev == total - 1) {
            *E.done = 0;
            __threadfence();
            *E.step = step + 1;
        }
    }
}

void launch_emt_history3(const EmtDev& E, const RecParams* rec, hipStream_t s)
{
    hipLaunchKernelGGL(k_emt_history3, dim3((E.n + kBlock - 1) / kBlock, E.n_cases), dim3(kBlock), 0, s, E, rec);
}

// Re-assemble b of the current step for case k from the stored histories,
// after a line loss was added for this step: b_a = i_in,a(t_n) - sum_e A[a,e] h_e^n
// - hC_a^n, with lost branches contributing nothing (same operation order as
// k_emt_history, so the result equals a loss scheduled in advance).
__global__ __launch_bounds__(kBlock) void k_emt_rebuild_rhs(EmtDev E, int k)
{
    const int64_t step = *E.step;
    const int64_t base = (int64_t)k * E.n;
    double* hcur = E.h + (int64_t)(step & 1) * E.n_cases * E.nbr + (int64_t)k * E.nbr;
    for (int a = blockIdx.x * kBlock + threadIdx.x; a < E.n; a += gridDim.x * kBlock) {
        double bn = source_at(E, a, (double)step * E.dt);
        for (int q = E.inc_ptr[a]; q < E.inc_ptr[a + 1]; ++q) {
            const int e = E.inc_br[q];
            const int f = E.fr[e];
            const double hn = lost_by(E, k, e, step) ? 0.0 : hcur[e];
            bn -= (a == f) ? hn : -hn;
        }
        bn -= E.hC[base + a];
        E.b[base + a] = bn;
    }
}

void launch_emt_rebuild_rhs(const EmtDev& E, int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_emt_rebuild_rhs, dim3((E.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, E, k);
}

__global__ void k_set_rec(RecParams* d, RecParams val) { *d = val; }

void launch_set_rec(RecParams* d, const RecParams& val, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_rec, dim3(1), dim3(1), 0, s, d, val);
}

}  // namespace hinv
