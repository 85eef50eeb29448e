// probe.hip -- microbenchmarks of the MI355X primitives the profitability
// model prices (the analogue of the paper's primitive-cost table, Sec. III-A,
// Table II): local (LDS) access latency and rates, the latency of the
// device-memory path the split-row exchange uses (L2 hit within an XCD, and a
// one-way handoff between workgroups on the same or on different XCDs), the
// workgroup barrier, and one exchange round of a row group of k workgroups.
//
// Every wait is bounded: a handoff that does not arrive within the spin limit
// sets the result's error word and the kernel returns.
#include "device.h"

namespace credit {

struct ProbeOut {
    unsigned long long cycles;  // s_memtime delta measured by the timing lane
    unsigned long long ticks;   // s_memrealtime delta (100 MHz) over the same span
    unsigned err;               // nonzero: a bounded wait gave up
    unsigned xcc[2];            // XCD of the two ping-pong workgroups
    unsigned sink;
};

__device__ __forceinline__ unsigned long long cyc() { return __builtin_readcyclecounter(); }
__device__ __forceinline__ unsigned long long rt() { return __builtin_amdgcn_s_memrealtime(); }
__device__ __forceinline__ unsigned xcc_id() {
    // HW_REG_XCC_ID (id 20), bits [3:0]: the XCD this wave runs on
    return __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11));
}

// LDS pointer chase: one lane follows `steps` dependent LDS loads.
__global__ __launch_bounds__(64) void k_probe_lds_latency(ProbeOut *o, int steps) {
    __shared__ unsigned nxt[4096];
    for (int i = threadIdx.x; i < 4096; i += 64) nxt[i] = (unsigned)((i * 1031 + 17) & 4095);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned p = 0;
        const unsigned long long c0 = cyc(), t0 = rt();
        for (int s = 0; s < steps; ++s) p = nxt[p];
        const unsigned long long c1 = cyc(), t1 = rt();
        o->cycles = c1 - c0;
        o->ticks = t1 - t0;
        o->sink = p;
    }
}

// Device-memory pointer chase with agent-scope loads (served by L2, bypassing
// the vector L1): the chain lives in a 64 KiB buffer, warmed by one pass.
__global__ __launch_bounds__(64) void k_probe_l2_latency(ProbeOut *o, const unsigned *chain, int steps) {
    if (threadIdx.x != 0) return;
    unsigned p = 0;
    for (int s = 0; s < 16384; ++s) p = __hip_atomic_load(chain + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long c0 = cyc(), t0 = rt();
    for (int s = 0; s < steps; ++s) p = __hip_atomic_load(chain + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long c1 = cyc(), t1 = rt();
    o->cycles = c1 - c0;
    o->ticks = t1 - t0;
    o->sink = p;
}

// Ping-pong between workgroups `a` and `b` of the grid through one word with
// agent-scope atomic stores and loads (the exchange's access path).  Round r:
// a writes 2r + 1 and waits for 2r + 2, which b writes once it has seen
// 2r + 1.  Round 0 only brings both up; a times rounds 1..rounds.  Other
// workgroups exit at once.
__device__ __forceinline__ bool wait_word(unsigned *word, unsigned want, unsigned spin_limit, ProbeOut *o) {
    unsigned spins = 0;
    while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
        if (++spins > spin_limit || __hip_atomic_load(&o->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
            __hip_atomic_store(&o->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

__global__ __launch_bounds__(64) void k_probe_pingpong(ProbeOut *o, unsigned *word, int a, int b, int rounds,
                                                       unsigned spin_limit) {
    const int bid = blockIdx.x;
    if ((bid != a && bid != b) || threadIdx.x != 0) return;
    const bool ping = bid == a;
    o->xcc[ping ? 0 : 1] = xcc_id();
    unsigned long long c0 = 0, t0 = 0;
    for (int r = 0; r <= rounds; ++r) {
        const unsigned v = 2u * (unsigned)r;
        if (ping) {
            __hip_atomic_store(word, v + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!wait_word(word, v + 2u, spin_limit, o)) return;
            if (r == 0) {
                c0 = cyc();
                t0 = rt();
            }
        } else {
            if (!wait_word(word, v + 1u, spin_limit, o)) return;
            __hip_atomic_store(word, v + 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (ping) {
        o->cycles = cyc() - c0;
        o->ticks = rt() - t0;
    }
}

// Workgroup barrier of 256 threads: `steps` back-to-back barriers.
__global__ __launch_bounds__(256) void k_probe_barrier(ProbeOut *o, int steps) {
    __shared__ unsigned v[256];
    v[threadIdx.x] = threadIdx.x;
    __syncthreads();
    const unsigned long long c0 = cyc(), t0 = rt();
    unsigned acc = 0;
    for (int s = 0; s < steps; ++s) {
        __syncthreads();
        acc += v[(threadIdx.x + s) & 255];
    }
    __syncthreads();
    const unsigned long long c1 = cyc(), t1 = rt();
    if (threadIdx.x == 0) {
        o->cycles = c1 - c0;
        o->ticks = t1 - t0;
        o->sink = acc;
    }
}

// One exchange round of a row group of k workgroups (the split-row kernel's
// exchange with q = 1), repeated for `rows` rows; workgroup 0 times it.
__global__ __launch_bounds__(kBlock) void k_probe_exchange(ProbeOut *o, RowArgs a, int rows) {
    __shared__ float xb[kMaxK * kMaxQ];
    const int c = blockIdx.x;
    __syncthreads();
    const unsigned long long c0 = cyc(), t0 = rt();
    float acc = 0.f;
    for (int r = 0; r < rows; ++r) {
        float mine[1] = {(float)(c + r)};
        exchange<1>(a, r, 0, c, mine, xb);
        acc += xb[(r + threadIdx.x) % a.k];
    }
    const unsigned long long c1 = cyc(), t1 = rt();
    if (c == 0 && threadIdx.x == 0) {
        o->cycles = c1 - c0;
        o->ticks = t1 - t0;
        o->sink = (unsigned)acc;
    }
}

// Streaming rates of one workgroup (256 threads, 16-byte accesses):
// kind 0 LDS read, 1 LDS write, 2 global read of an L2-resident 256 KiB
// buffer, 3 global write of the same buffer.  `reps` passes over the region.
__global__ __launch_bounds__(256) void k_probe_rate(ProbeOut *o, u32x4 *buf, int kind, int reps) {
    __shared__ u32x4 lds[2048];  // 32 KiB
    const int t = threadIdx.x;
    for (int i = t; i < 2048; i += 256) lds[i] = u32x4{(unsigned)i, 0u, 0u, 0u};
    __syncthreads();
    u32x4 acc = {0u, 0u, 0u, 0u};
    if (kind == 2)
        for (int i = t; i < 16384; i += 256) acc ^= buf[i];  // warm the L2 (256 KiB: past the vector L1)
    __syncthreads();
    const unsigned long long c0 = cyc(), t0 = rt();
    for (int r = 0; r < reps; ++r) {
        if (kind == 0) {
#pragma unroll 8
            for (int i = t; i < 2048; i += 256) acc ^= lds[(i + r) & 2047];
        } else if (kind == 1) {
#pragma unroll 8
            for (int i = t; i < 2048; i += 256) lds[i] = u32x4{(unsigned)r, (unsigned)i, 0u, 0u};
        } else if (kind == 2) {
#pragma unroll 8
            for (int i = t; i < 16384; i += 256) acc ^= buf[(i + 256 * r) & 16383];
        } else {
#pragma unroll 8
            for (int i = t; i < 16384; i += 256) buf[i] = u32x4{(unsigned)r, (unsigned)i, 0u, 0u};
        }
    }
    __syncthreads();
    const unsigned long long c1 = cyc(), t1 = rt();
    if (t == 0) {
        o->cycles = c1 - c0;
        o->ticks = t1 - t0;
        o->sink = acc[0] ^ acc[1] ^ lds[(reps + 5) & 2047][1];
    }
}

const void *probe_kernel(int which) {
    switch (which) {
    case 0: return (const void *)&k_probe_lds_latency;
    case 1: return (const void *)&k_probe_l2_latency;
    case 2: return (const void *)&k_probe_pingpong;
    case 3: return (const void *)&k_probe_barrier;
    case 4: return (const void *)&k_probe_exchange;
    case 5: return (const void *)&k_probe_rate;
    }
    return nullptr;
}

}  // namespace credit
