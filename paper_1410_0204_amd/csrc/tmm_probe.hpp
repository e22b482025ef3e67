// Latency probes of the primitives the persistent kernels chain in every time
// step: an agent-scope store seen by an agent-scope poll in another
// workgroup (the state exchange), a workgroup barrier, and a dependent
// agent-scope load.  They give the floor below which a step that hands its
// state to a neighbouring domain cannot go, whatever its arithmetic.
//
// Every wait is bounded (kProbeMaxPolls polls); a wait that gives up sets
// *fail and returns, and its partner then gives up too, so every launch ends.
#pragma once

#include <hip/hip_runtime.h>

namespace tmm {

constexpr long long kProbeMaxPolls = 1ll << 24;
constexpr int kProbeWordStride = 32;      // 256 bytes between the two ping-pong words

__device__ __forceinline__ int xcc_id() {
    int x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x & 0xf;
}

// Round trips between workgroups a and b (lane 0 of each): in round r, a
// stores r to word 0 and polls word 1 for r; b polls word 0 for r and stores
// r to word 1.  Stores and polls are the persistent kernels' (relaxed, agent
// scope, one s_sleep between polls).  out[0] = ticks of a's loop, out[1..2] =
// the XCDs a and b ran on.  words[0] and words[kProbeWordStride] must be 0.
__global__ void k_probe_pingpong(int a, int b, int rounds, long long* __restrict__ words,
                                 long long* __restrict__ out, int* __restrict__ fail) {
    if ((int)blockIdx.x != a && (int)blockIdx.x != b) return;
    if (threadIdx.x != 0) return;
    const bool ping = (int)blockIdx.x == a;
    long long* mine = ping ? words : words + kProbeWordStride;
    long long* theirs = ping ? words + kProbeWordStride : words;
    out[ping ? 1 : 2] = xcc_id();
    const long long t0 = wall_clock64();
    for (long long r = 1; r <= rounds; ++r) {
        if (ping) __hip_atomic_store(mine, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        long long it = 0;
        while (__hip_atomic_load(theirs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < r) {
            if (++it > kProbeMaxPolls ||
                ((it & 63) == 0 && __hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!ping) __hip_atomic_store(mine, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (ping) out[0] = wall_clock64() - t0;
}

// Workgroup barriers with one LDS write between them, as in a time step.
// out[0] = ticks for n barriers.
template <int TPB>
__global__ __launch_bounds__(TPB) void k_probe_barrier(int n, long long* __restrict__ out) {
    __shared__ double s[TPB];
    s[threadIdx.x] = 0.0;
    __syncthreads();
    const long long t0 = wall_clock64();
    for (int i = 0; i < n; ++i) {
        s[(threadIdx.x + i) % TPB] += 1.0;
        __syncthreads();
    }
    const long long t1 = wall_clock64();
    if (threadIdx.x == 0) out[0] = t1 - t0 + (s[0] > 1e300 ? 1 : 0);
}

// A chain of n dependent agent-scope loads through next[] (a cycle over
// distinct 256-byte lines).  out[0] = ticks.
__global__ void k_probe_load(int n, const int* __restrict__ next, long long* __restrict__ out) {
    if (threadIdx.x != 0) return;
    int i = 0;
    const long long t0 = wall_clock64();
    for (int k = 0; k < n; ++k) i = __hip_atomic_load(&next[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    out[0] = wall_clock64() - t0 + (i < 0 ? 1 : 0);
}

// next[l * 64] = ((l + step) % nlines) * 64: a cycle over nlines lines of 256 bytes.
__global__ void k_probe_chain(int nlines, int step, int* __restrict__ next) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nlines) next[(size_t)l * 64] = ((l + step) % nlines) * 64;
}

}  // namespace tmm
