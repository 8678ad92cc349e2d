// Barrier among the T workgroups of one team (cooperative launches of the
// team and panel engines), by per-workgroup epoch flags: each workgroup
// release-stores its epoch after all its threads' global writes, one
// wavefront polls every flag of the team with relaxed agent-scope loads and a
// wave vote, and a single acquire fence follows; there is no read-modify-write
// on a shared counter.  The wait is bounded: on time-out the barrier raises
// kFlagBarrier in *errflags and returns false in every thread.
#pragma once
#include "hinv_internal.h"

namespace hinv {

constexpr int kTeamSpinLimit = 1 << 24;

// flags: the team's T flags; me: this workgroup's flag; ctl: one int of LDS.
__device__ inline bool team_barrier(unsigned int* flags, int me, int T, unsigned int epoch, int* errflags, int* ctl)
{
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&flags[me], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
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
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (threadIdx.x == 0) {
            ctl[0] = ok;
            if (!ok) atomicOr(errflags, kFlagBarrier);
        }
    }
    __syncthreads();
    return ctl[0] != 0;
}

}  // namespace hinv
