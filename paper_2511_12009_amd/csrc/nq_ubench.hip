// Microbenchmarks behind the DFS kernel's roofline: the int32 VALU issue rate
// of the operations its step is made of, and the LDS cost of its stack
// accesses in the lane-interleaved layout against a per-lane contiguous one.
//
// VALU: every lane runs `chains` independent dependency chains of one
// operation (v_add3_u32, v_bitop3_b32, v_cndmask_b32 with an SGPR lane mask,
// v_addc_co_u32 with an SGPR carry-in, v_add_lshl_u32, v_xad_u32), `iters`
// operations per chain, in 1..8 single-wave workgroups per SIMD.  With eight
// chains a wave has eight independent instructions in flight and the SIMD's
// issue rate shows; with one chain the dependent latency shows.  Each wave
// also records its shader-clock cycles (s_memtime), so the clock during the
// run and the cycles per instruction come out of the same launch.
//
// LDS: each lane keeps a stack position and per iteration writes one 16-byte
// frame and reads one back (ds_write_b128 / ds_read_b128), at per-lane
// positions that differ across the wave, in either layout: interleaved (frame
// f of lane l at (f * 64 + l) * 16, as the DFS kernel's stack) or contiguous
// (lane l's frames at (l * frames + f) * 16).  `active` lanes of each wave take
// part (the rest are masked off, as lanes that do not push or pop in a step).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nq_internal.h"
#include "../../include/nq_ubench.h"

namespace nqi {

namespace {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

template <int OP>
__device__ __forceinline__ void valu_op(uint32_t& d, uint32_t b, uint32_t c, uint64_t m) {
    if (OP == 0) {
        asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(d) : "v"(b), "v"(c));
    } else if (OP == 1) {
        asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(d) : "v"(b), "v"(c));
    } else if (OP == 2) {
        asm volatile("v_cndmask_b32 %0, %0, %1, %2" : "+v"(d) : "v"(b), "s"(m));
    } else if (OP == 3) {
        uint64_t junk;
        asm volatile("v_addc_co_u32 %0, %1, %0, %2, %3" : "+v"(d), "=s"(junk) : "v"(b), "s"(m));
    } else if (OP == 4) {
        asm volatile("v_add_lshl_u32 %0, %0, %1, 1" : "+v"(d) : "v"(b));
    } else if (OP == 5) {
        asm volatile("v_xad_u32 %0, %0, %1, %2" : "+v"(d) : "v"(b), "v"(c));
    } else if (OP == 6) {
        asm volatile("v_and_b32 %0, %0, %1" : "+v"(d) : "v"(b));
    } else if (OP == 7) {
        asm volatile("v_xor_b32 %0, %0, %1" : "+v"(d) : "v"(b));
    } else if (OP == 8) {
        asm volatile("v_or3_b32 %0, %0, %1, %2" : "+v"(d) : "v"(b), "v"(c));
    } else if (OP == 9) {
        asm volatile("v_sub_u32 %0, %1, %0" : "+v"(d) : "v"(b));
    } else if (OP == 10) {
        asm volatile("v_lshrrev_b32 %0, 1, %0" : "+v"(d));
    } else {
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(d) : "v"(b));
    }
}

// `iters` is a multiple of 8; each trip issues 8 operations per chain.
template <int OP, int CHAINS>
__global__ __launch_bounds__(64) void ubench_valu_kernel(uint64_t iters, uint32_t seed,
                                                         uint32_t* sink, uint64_t* cycles) {
    const uint32_t lane = threadIdx.x;
    uint32_t d[CHAINS];
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) d[i] = seed * (lane + 1u) + 0x9e3779b9u * (uint32_t)i;
    const uint32_t b = seed ^ lane, c = seed + 7u * lane;
    const uint64_t m = __builtin_amdgcn_ballot_w64((lane & 3u) != 0u);
    const uint64_t t0 = __builtin_amdgcn_s_memtime();
    for (uint64_t it = 0; it < iters; it += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
#pragma unroll
            for (int i = 0; i < CHAINS; ++i) valu_op<OP>(d[i], b, c, m);
        }
    }
    const uint64_t t1 = __builtin_amdgcn_s_memtime();
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) x ^= d[i];
    sink[blockIdx.x * 64u + lane] = x;
    if (lane == 0) cycles[blockIdx.x] = t1 - t0;
}

// One iteration's LDS accesses at byte addresses wa (write) and ra (read), by
// op: 0 = write b128 + read b128, 1 = read b128, 2 = write b128, 3 = one
// 16-byte exchange (ds_wrxchg2_rtn_b64 of two adjacent qwords at wa), 4 =
// write b64 + read b64, 5 = write b32 + read b32, 6 = write b64, 7 = write
// b32, 8 = write b96, 9 = 16 bytes as ds_write2_b64 (two adjacent qwords),
// 10 = read b96, 11 = 16 bytes as ds_read2_b64, 12 = write b96 + read b96 (a
// 12-byte frame in the same 16-byte slots).
template <int OP>
__device__ __forceinline__ void lds_op(v4u& v, int32_t wa, int32_t ra) {
    if (OP == 0) {
        asm volatile("ds_write_b128 %[wa], %[v]\n\tds_read_b128 %[v], %[ra]\n\ts_waitcnt lgkmcnt(0)"
                     : [v] "+v"(v) : [wa] "v"(wa), [ra] "v"(ra) : "memory");
    } else if (OP == 1) {
        asm volatile("ds_read_b128 %[v], %[ra]\n\ts_waitcnt lgkmcnt(0)"
                     : [v] "+v"(v) : [ra] "v"(ra) : "memory");
    } else if (OP == 2) {
        asm volatile("ds_write_b128 %[wa], %[v]\n\ts_waitcnt lgkmcnt(0)"
                     : : [v] "v"(v), [wa] "v"(wa) : "memory");
        v.w += 1u;
    } else if (OP == 3) {
        const uint64_t lo = ((uint64_t)v.y << 32) | v.x, hi = ((uint64_t)v.w << 32) | v.z;
        v4u r;
        asm volatile("ds_wrxchg2_rtn_b64 %[r], %[wa], %[lo], %[hi] offset1:1\n\ts_waitcnt lgkmcnt(0)"
                     : [r] "=&v"(r) : [wa] "v"(wa), [lo] "v"(lo), [hi] "v"(hi) : "memory");
        v = r;
        v.w += 1u;
    } else if (OP == 4) {
        uint64_t x = ((uint64_t)v.y << 32) | v.x;
        asm volatile("ds_write_b64 %[wa], %[x]\n\tds_read_b64 %[x], %[ra]\n\ts_waitcnt lgkmcnt(0)"
                     : [x] "+v"(x) : [wa] "v"(wa), [ra] "v"(ra) : "memory");
        v.x = (uint32_t)x;
        v.y = (uint32_t)(x >> 32);
        v.w += v.x;
    } else if (OP == 5) {
        asm volatile("ds_write_b32 %[wa], %[x]\n\tds_read_b32 %[x], %[ra]\n\ts_waitcnt lgkmcnt(0)"
                     : [x] "+v"(v.x) : [wa] "v"(wa), [ra] "v"(ra) : "memory");
        v.w += v.x;
    } else if (OP == 6) {
        const uint64_t x = ((uint64_t)v.y << 32) | v.x;
        asm volatile("ds_write_b64 %[wa], %[x]\n\ts_waitcnt lgkmcnt(0)"
                     : : [x] "v"(x), [wa] "v"(wa) : "memory");
        v.w += 1u;
    } else if (OP == 7) {
        asm volatile("ds_write_b32 %[wa], %[x]\n\ts_waitcnt lgkmcnt(0)"
                     : : [x] "v"(v.x), [wa] "v"(wa) : "memory");
        v.w += 1u;
    } else if (OP == 8) {
        typedef uint32_t v3u __attribute__((ext_vector_type(3)));
        const v3u x = {v.x, v.y, v.z};
        asm volatile("ds_write_b96 %[wa], %[x]\n\ts_waitcnt lgkmcnt(0)"
                     : : [x] "v"(x), [wa] "v"(wa) : "memory");
        v.w += 1u;
    } else if (OP == 9) {
        const uint64_t lo = ((uint64_t)v.y << 32) | v.x, hi = ((uint64_t)v.w << 32) | v.z;
        asm volatile("ds_write2_b64 %[wa], %[lo], %[hi] offset1:1\n\ts_waitcnt lgkmcnt(0)"
                     : : [lo] "v"(lo), [hi] "v"(hi), [wa] "v"(wa) : "memory");
        v.w += 1u;
    } else if (OP == 10) {
        typedef uint32_t v3u __attribute__((ext_vector_type(3)));
        v3u x;
        asm volatile("ds_read_b96 %[x], %[ra]\n\ts_waitcnt lgkmcnt(0)"
                     : [x] "=v"(x) : [ra] "v"(ra) : "memory");
        v.x = x.x; v.y = x.y; v.z = x.z;
    } else if (OP == 11) {
        v4u x;
        asm volatile("ds_read2_b64 %[x], %[ra] offset1:1\n\ts_waitcnt lgkmcnt(0)"
                     : [x] "=v"(x) : [ra] "v"(ra) : "memory");
        v = x;
    } else {
        typedef uint32_t v3u __attribute__((ext_vector_type(3)));
        v3u x = {v.x, v.y, v.z};
        asm volatile("ds_write_b96 %[wa], %[x]\n\tds_read_b96 %[x], %[ra]\n\ts_waitcnt lgkmcnt(0)"
                     : [x] "+v"(x) : [wa] "v"(wa), [ra] "v"(ra) : "memory");
        v.x = x.x; v.y = x.y; v.z = x.z;
        v.w += v.x;
    }
}

template <int OP>
__global__ __launch_bounds__(64) void ubench_lds_kernel(uint32_t layout, uint32_t frames,
                                                        uint32_t active, uint64_t iters,
                                                        uint32_t* sink) {
    extern __shared__ v4u lds_frames[];
    const uint32_t lane = threadIdx.x;
    const int32_t base = (int32_t)(uint32_t)(uintptr_t)(__attribute__((address_space(3))) v4u*)lds_frames;
    // the byte offset of frame f of this lane, and the step between frames
    const int32_t lane_off = layout == 0 ? (int32_t)(lane * 16u) : (int32_t)(lane * frames * 16u);
    const int32_t stride = layout == 0 ? 1024 : 16;
    uint32_t f = (lane * 5u) % frames;
    v4u v = {lane, lane ^ 0x5a5a5a5au, lane * 3u, 1u};
    uint32_t acc = 0;
    if (lane < active) {
        for (uint64_t it = 0; it < iters; ++it) {
            const int32_t wa = base + lane_off + (int32_t)f * stride;
            uint32_t g = f + 1u + (v.w & 1u);                     // data-dependent next level
            g = g >= frames ? g - frames : g;
            const int32_t ra = base + lane_off + (int32_t)g * stride;
            lds_op<OP>(v, wa, ra);
            acc += v.x;
            f = g;
        }
    }
    sink[blockIdx.x * 64u + lane] = acc + v.y;
}

template <int OP>
const void* valu_kernel(uint32_t chains) {
    return chains == 1 ? reinterpret_cast<const void*>(&ubench_valu_kernel<OP, 1>)
                       : reinterpret_cast<const void*>(&ubench_valu_kernel<OP, 8>);
}

const void* pick_valu(uint32_t op, uint32_t chains) {
    switch (op) {
        case 0: return valu_kernel<0>(chains);
        case 1: return valu_kernel<1>(chains);
        case 2: return valu_kernel<2>(chains);
        case 3: return valu_kernel<3>(chains);
        case 4: return valu_kernel<4>(chains);
        case 5: return valu_kernel<5>(chains);
        case 6: return valu_kernel<6>(chains);
        case 7: return valu_kernel<7>(chains);
        case 8: return valu_kernel<8>(chains);
        case 9: return valu_kernel<9>(chains);
        case 10: return valu_kernel<10>(chains);
        default: return valu_kernel<11>(chains);
    }
}

// Runs `fn` on grid x 64 threads with `lds` bytes of dynamic LDS and returns
// the event time of the launch; `args` are the kernel's arguments.
int timed_launch(const void* fn, uint32_t grid, uint32_t lds, void** args, double* ms) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
        set_hip_error(e);
        if (a) (void)hipEventDestroy(a);
        return NQ_EDEVICE;
    }
    float f = 0.f;
    e = hipEventRecord(a, nullptr);
    if (e == hipSuccess) e = hipLaunchKernel(fn, dim3(grid), dim3(64), args, lds, nullptr);
    if (e == hipSuccess) e = hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    *ms = f;
    return NQ_OK;
}

}  // namespace

}  // namespace nqi

using namespace nqi;

extern "C" int nq_ubench_valu(uint32_t op, uint32_t chains, uint32_t waves_per_simd,
                              uint64_t iters, double* kernel_ms, double* mean_cycles) {
    if (op > 11 || (chains != 1 && chains != 8) || waves_per_simd < 1 || waves_per_simd > 8 ||
        iters == 0 || iters % 8 != 0 || !kernel_ms || !mean_cycles)
        return NQ_EINVAL;
    DeviceInfo dev;
    int rc = device_info(&dev);
    if (rc != NQ_OK) return rc;
    const uint32_t grid = (uint32_t)dev.cu_count * 4u * waves_per_simd;
    uint32_t* sink = nullptr;
    uint64_t* cyc = nullptr;
    hipError_t e = hipMalloc((void**)&sink, (size_t)grid * 64 * 4);
    if (e == hipSuccess) e = hipMalloc((void**)&cyc, (size_t)grid * 8);
    if (e != hipSuccess) {
        set_hip_error(e);
        if (sink) (void)hipFree(sink);
        return NQ_EDEVICE;
    }
    uint32_t seed = 0x2511u;
    void* args[] = {&iters, &seed, &sink, &cyc};
    double ms = 0.0;
    rc = timed_launch(pick_valu(op, chains), grid, 0, args, &ms);
    std::vector<uint64_t> host(grid);
    if (rc == NQ_OK) {
        e = hipMemcpy(host.data(), cyc, (size_t)grid * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) { set_hip_error(e); rc = NQ_EDEVICE; }
    }
    (void)hipFree(sink);
    (void)hipFree(cyc);
    if (rc != NQ_OK) return rc;
    double sum = 0.0;
    for (uint64_t c : host) sum += (double)c;
    *kernel_ms = ms;
    *mean_cycles = sum / grid;
    return NQ_OK;
}

extern "C" int nq_ubench_lds(uint32_t layout, uint32_t op, uint32_t active_lanes,
                             uint32_t waves_per_cu, uint32_t frames, uint64_t iters,
                             double* kernel_ms) {
    if (layout > 1 || op > 12 || active_lanes < 1 || active_lanes > 64 || waves_per_cu < 1 ||
        waves_per_cu > 32 || frames < 2 || frames > 32 || iters == 0 || !kernel_ms)
        return NQ_EINVAL;
    DeviceInfo dev;
    int rc = device_info(&dev);
    if (rc != NQ_OK) return rc;
    const uint32_t lds = frames * 64u * 16u;
    if ((uint64_t)lds * waves_per_cu > (uint64_t)dev.lds_per_cu) return NQ_EINVAL;
    const uint32_t grid = (uint32_t)dev.cu_count * waves_per_cu;
    uint32_t* sink = nullptr;
    hipError_t e = hipMalloc((void**)&sink, (size_t)grid * 64 * 4);
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    void* args[] = {&layout, &frames, &active_lanes, &iters, &sink};
    const void* fns[] = {reinterpret_cast<const void*>(&ubench_lds_kernel<0>),
                         reinterpret_cast<const void*>(&ubench_lds_kernel<1>),
                         reinterpret_cast<const void*>(&ubench_lds_kernel<2>),
                         reinterpret_cast<const void*>(&ubench_lds_kernel<3>),
                         reinterpret_cast<const void*>(&ubench_lds_kernel<4>),
                         reinterpret_cast<const void*>(&ubench_lds_kernel<5>),
                         reinterpret_cast<const void*>(&ubench_lds_kernel<6>),
                         reinterpret_cast<const void*>(&ubench_lds_kernel<7>),
                         reinterpret_cast<const void*>(&ubench_lds_kernel<8>),
                         reinterpret_cast<const void*>(&ubench_lds_kernel<9>),
                         reinterpret_cast<const void*>(&ubench_lds_kernel<10>),
                         reinterpret_cast<const void*>(&ubench_lds_kernel<11>),
                         reinterpret_cast<const void*>(&ubench_lds_kernel<12>)};
    double ms = 0.0;
    rc = timed_launch(fns[op], grid, lds, args, &ms);
    (void)hipFree(sink);
    if (rc != NQ_OK) return rc;
    *kernel_ms = ms;
    return NQ_OK;
}
