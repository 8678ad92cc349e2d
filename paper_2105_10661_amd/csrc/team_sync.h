// Barrier among the T workgroups of one team (cooperative launches of the
// team and panel engines), by per-workgroup epoch flags, and the accessors of
// the data the workgroups exchange through global memory.
//
// Every value that one workgroup writes for another is stored and loaded with
// device-scope ("agent") relaxed atomics (xchg_store / xchg_load).  Those are
// coherent at device scope without the per-XCD L2 (stores complete at the
// device coherence point, loads are served from it), so the barrier needs no
// L2 write-back or invalidate: each wavefront waits until its stores have
// completed (vmcnt(0)), the workgroup synchronises, one thread stores the
// epoch flag, one wavefront polls the team's flags (relaxed device-scope
// loads and a wave vote), and the workgroup synchronises again before any
// exchanged value is loaded.  The wait is bounded: on time-out the barrier
// raises kFlagBarrier in *errflags and returns false in every thread.
#pragma once
#include "hinv_internal.h"

namespace hinv {

constexpr int kTeamSpinLimit = 1 << 24;

__device__ __forceinline__ void xchg_store(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double xchg_load(const double* p)
{
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tagged exchange of one FP64 value without a barrier: the value's low and high 32 bits, each in
// one 64-bit word under a 32-bit tag, stored and loaded as 64-bit device-scope relaxed atomics, so a
// reader sees each half together with its tag.  A value is read once both words carry the expected
// tag.  The wait is bounded: on time-out *ok is cleared and 0 is returned.
__device__ __forceinline__ void tagged_store(unsigned long long* p, double v, unsigned int tag)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned long long t = (unsigned long long)tag << 32;
    __hip_atomic_store(p, t | (b & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, t | (b >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double tagged_load(unsigned long long* p, unsigned int tag, bool* ok)
{
    for (int spins = 0;; ++spins) {
        const unsigned long long w0 = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long w1 = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((unsigned int)(w0 >> 32) == tag && (unsigned int)(w1 >> 32) == tag)
            return __longlong_as_double((long long)((w1 << 32) | (w0 & 0xffffffffull)));
        if (spins >= kTeamSpinLimit) {
            *ok = false;
            return 0.0;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Value of another lane of the same quad (lanes 4q .. 4q + 3) by a DPP quad permutation: a VALU
// move, no LDS round trip.  CTRL 0xB1 = quad_perm [1,0,3,2] (lane ^ 1), 0x4E = [2,3,0,1] (lane ^ 2).
template <int CTRL>
__device__ __forceinline__ double quad_mov(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float quad_mov(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the four lanes of a quad, all four active: (a + a[^1]) + (...)[^2], every lane gets it.
template <typename T>
__device__ __forceinline__ T quad_sum(T a)
{
    a += quad_mov<0xB1>(a);
    a += quad_mov<0x4E>(a);
    return a;
}

// Value of lane 7 - i of the same eight lanes (DPP row_half_mirror, 0x141): after quad_sum, adding
// it gives the sum over the eight lanes in every one of them.
__device__ __forceinline__ double half_row_mirror(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x141, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x141, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float half_row_mirror(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
}

// Sum over eight consecutive lanes (aligned), all eight active: every lane gets it.
template <typename T>
__device__ __forceinline__ T oct_sum(T a)
{
    a = quad_sum(a);
    return a + half_row_mirror(a);
}

// The barrier in two halves, so that a workgroup can do work that no other workgroup waits for
// while its wavefront 0 polls.  team_arrive: this workgroup's stores have completed, then its flag
// is raised (flags: the team's T flags; me: this workgroup's flag).
__device__ inline void team_arrive(unsigned int* flags, int me, unsigned int epoch)
{
    __builtin_amdgcn_s_waitcnt(0x0F70);   // gfx9 encoding of vmcnt(0): this wave's stores have completed
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&flags[me], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// team_wait: wavefront 0 polls the team's flags (bounded), then the workgroup synchronises; ctl: one
// int of LDS.  Returns false in every thread on time-out.
__device__ inline bool team_wait(unsigned int* flags, int T, unsigned int epoch, int* errflags, int* ctl)
{
    if (threadIdx.x < 64) {
        int ok = 1;
        int spins = 0;
        while (true) {
            int mine = 1;
            for (int i = threadIdx.x; i < T; i += 64)
                mine &= (__hip_atomic_load(&flags[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch) ? 1 : 0;
            if (__all(mine)) break;
            if (++spins > kTeamSpinLimit) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (threadIdx.x == 0) {
            ctl[0] = ok;
            if (!ok) atomicOr(errflags, kFlagBarrier);
        }
    }
    __syncthreads();
    return ctl[0] != 0;
}

__device__ inline bool team_barrier(unsigned int* flags, int me, int T, unsigned int epoch, int* errflags, int* ctl)
{
    team_arrive(flags, me, epoch);
    return team_wait(flags, T, epoch, errflags, ctl);
}

// Barrier of a large team by one arrival counter (counter: one word, zero at the launch; epoch:
// 1, 2, ... per barrier of the launch).  Each workgroup's stores complete, then one thread adds 1
// and polls the single word until all T workgroups of this epoch have arrived (epoch * T).  With
// one flag per workgroup, a team of 128 polls 128 words from every workgroup (16K device-scope
// loads per round); the counter costs T atomic adds and one word per poll.  Bounded like team_wait.
// The counter barrier in two halves (as team_arrive / team_wait).
__device__ inline void count_arrive(unsigned int* counter)
{
    __builtin_amdgcn_s_waitcnt(0x0F70);   // gfx9 encoding of vmcnt(0): this wave's stores have completed
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline bool count_wait(unsigned int* counter, int T, unsigned int epoch, int* errflags, int* ctl)
{
    if (threadIdx.x == 0) {
        const unsigned int target = epoch * (unsigned int)T;
        int ok = 1;
        int spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kTeamSpinLimit) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        ctl[0] = ok;
        if (!ok) atomicOr(errflags, kFlagBarrier);
    }
    __syncthreads();
    return ctl[0] != 0;
}

__device__ inline bool count_barrier(unsigned int* counter, int T, unsigned int epoch, int* errflags, int* ctl)
{
    __builtin_amdgcn_s_waitcnt(0x0F70);   // gfx9 encoding of vmcnt(0): this wave's stores have completed
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned int target = epoch * (unsigned int)T;
        int ok = 1;
        int spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kTeamSpinLimit) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        ctl[0] = ok;
        if (!ok) atomicOr(errflags, kFlagBarrier);
    }
    __syncthreads();
    return ctl[0] != 0;
}

}  // namespace hinv
