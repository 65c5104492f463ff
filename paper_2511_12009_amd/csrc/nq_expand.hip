// Device frontier expansion: Algorithm 1 continued on the GPU.
//
// Given subproblems at depth k (Somers triples, Section 2), produce every
// placement of `rows` more queens below each of them, i.e. the frontier at
// depth k + rows, in canonical order: the children of entry i follow those of
// entry i - 1, and each entry's children are in lowest-column-first order, so
// expanding the depth-k frontier gives exactly nq_frontier(n, k + rows) for
// k >= 2 or even n.  Children inherit their parent's weight (for odd n from
// depth 1 the weight-1 centre entry keeps its unrestricted row 1, which gives
// the same weighted count as the deeper frontier's restricted, weight-2 form).
//
// Three passes: count the children of every entry (one thread per entry), an
// exclusive scan of the counts (rocPRIM via hipCUB) giving each entry's output
// offset, and the write pass.  The host builds a shallow frontier in
// milliseconds and the device produces the deep one at HBM speed.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "nq_internal.h"

namespace nqi {

namespace {

constexpr uint32_t kMaxExpandRows = 3;

// Visits the children `rows` rows below (c, l, r), lowest column first.
template <class Emit>
__device__ __forceinline__ void for_each_child(uint32_t last, uint32_t rows, uint32_t c,
                                               uint32_t l, uint32_t r, Emit&& emit) {
    uint32_t a0 = last & ~(c | l | r);
    while (a0) {
        const uint32_t p0 = a0 & (0u - a0);
        a0 ^= p0;
        const uint32_t c1 = c | p0, l1 = (l | p0) << 1, r1 = (r | p0) >> 1;
        if (rows == 1) { emit(c1, l1 & last, r1); continue; }
        uint32_t a1 = last & ~(c1 | l1 | r1);
        while (a1) {
            const uint32_t p1 = a1 & (0u - a1);
            a1 ^= p1;
            const uint32_t c2 = c1 | p1, l2 = (l1 | p1) << 1, r2 = (r1 | p1) >> 1;
            if (rows == 2) { emit(c2, l2 & last, r2); continue; }
            uint32_t a2 = last & ~(c2 | l2 | r2);
            while (a2) {
                const uint32_t p2 = a2 & (0u - a2);
                a2 ^= p2;
                emit(c2 | p2, ((l2 | p2) << 1) & last, (r2 | p2) >> 1);
            }
        }
    }
}

__global__ void nq_expand_count_kernel(const uint32_t* __restrict__ cols,
                                       const uint32_t* __restrict__ ld,
                                       const uint32_t* __restrict__ rd, uint64_t len,
                                       uint32_t n, uint32_t rows, uint64_t* __restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    const uint32_t last = (1u << n) - 1u;
    uint64_t k = 0;
    for_each_child(last, rows, cols[i] & last, ld[i] & last, rd[i] & last,
                   [&](uint32_t, uint32_t, uint32_t) { ++k; });
    out[i] = k;
}

// Write pass, one wave per 64 parents.  The wave's children form one
// contiguous range of the output (the offsets are a prefix sum), which is
// written in chunks of kChunk entries: every lane places the children of its
// parent that fall into the current chunk into LDS, then the wave stores the
// chunk with consecutive lanes on consecutive entries (coalesced), instead of
// each lane storing its own run of children with scattered 4-byte stores.
constexpr uint32_t kChunk = 1024;

__global__ __launch_bounds__(64) void nq_expand_write_kernel(
    const uint32_t* __restrict__ cols, const uint32_t* __restrict__ ld,
    const uint32_t* __restrict__ rd, const uint8_t* __restrict__ w, uint64_t len, uint32_t n,
    uint32_t rows, const uint64_t* __restrict__ offsets, uint32_t* __restrict__ ocols,
    uint32_t* __restrict__ old, uint32_t* __restrict__ ord, uint8_t* __restrict__ ow) {
    __shared__ uint32_t s_c[kChunk], s_l[kChunk], s_r[kChunk];
    __shared__ uint8_t s_w[kChunk];
    const uint64_t first = (uint64_t)blockIdx.x * 64u;
    const uint64_t i = first + threadIdx.x;
    const uint64_t last_parent = min(first + 64u, len);          // exclusive
    const uint64_t r0 = offsets[first], r1 = offsets[last_parent];
    const uint32_t mask = (1u << n) - 1u;
    const bool mine = i < len;
    const uint64_t o0 = mine ? offsets[i] : r1, o1 = mine ? offsets[i + 1] : r1;
    const uint32_t c = mine ? cols[i] & mask : 0u, l = mine ? ld[i] & mask : 0u,
                   r = mine ? rd[i] & mask : 0u;
    const uint8_t wt = (mine && w) ? w[i] : (uint8_t)1;
    for (uint64_t base = r0; base < r1; base += kChunk) {
        const uint64_t end = min(base + (uint64_t)kChunk, r1);
        if (o0 < end && o1 > base) {
            uint64_t o = o0;
            for_each_child(mask, rows, c, l, r, [&](uint32_t cc, uint32_t cl, uint32_t cr) {
                if (o >= base && o < end) {
                    const uint32_t t = (uint32_t)(o - base);
                    s_c[t] = cc;
                    s_l[t] = cl;
                    s_r[t] = cr;
                    s_w[t] = wt;
                }
                ++o;
            });
        }
        __syncthreads();
        const uint32_t m = (uint32_t)(end - base);
        for (uint32_t t = threadIdx.x; t < m; t += 64u) {
            ocols[base + t] = s_c[t];
            old[base + t] = s_l[t];
            ord[base + t] = s_r[t];
            if (ow) ow[base + t] = s_w[t];
        }
        __syncthreads();
    }
}

}  // namespace

// Enqueues the expansion on `stream`.  `scratch` must hold expand_scratch_bytes
// (len) bytes; the output arrays must hold `cap` entries.  *out_len (host) gets
// the child count, which requires a wait on the stream (done here).
size_t expand_scratch_bytes(uint64_t len) {
    size_t scan_bytes = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (const uint64_t*)nullptr,
                                           (uint64_t*)nullptr,
                                           (int)std::min<uint64_t>(len + 1, 0x7fffffff));
    return (len + 1) * 8 * 2 + scan_bytes + 256;
}

int expand_device(uint32_t n, uint32_t rows, const uint32_t* cols, const uint32_t* ld,
                  const uint32_t* rd, const uint8_t* w, uint64_t len, uint32_t* ocols,
                  uint32_t* old, uint32_t* ord, uint8_t* ow, uint64_t cap, uint64_t* out_len,
                  void* scratch, void* stream) {
    if (n < 1 || n > NQ_MAX_N_WIDE || rows < 1 || rows > kMaxExpandRows || !out_len) return NQ_EINVAL;
    if (len >= (uint64_t)0x7fffffff) return NQ_EINVAL;        // scan index range
    hipStream_t s = (hipStream_t)stream;
    if (len == 0) { *out_len = 0; return NQ_OK; }
    char* sc = static_cast<char*>(scratch);
    uint64_t* counts = reinterpret_cast<uint64_t*>(sc);
    uint64_t* offsets = counts + (len + 1);
    void* scan_tmp = offsets + (len + 1);
    size_t scan_bytes = 0;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, counts, offsets,
                                                    (int)(len + 1), s);
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    if (scan_bytes + (len + 1) * 16 + 256 > expand_scratch_bytes(len)) return NQ_EINVAL;
    const uint32_t block = 256;
    const uint32_t grid = (uint32_t)((len + block - 1) / block);
    // counts[len] = 0 so that offsets[len] is the total.
    int rc = launch_zero_u64(reinterpret_cast<unsigned long long*>(counts + len), 1, stream);
    if (rc != NQ_OK) return rc;
    hipLaunchKernelGGL(nq_expand_count_kernel, dim3(grid), dim3(block), 0, s, cols, ld, rd, len,
                       n, rows, counts);
    if ((e = hipGetLastError()) != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    e = hipcub::DeviceScan::ExclusiveSum(scan_tmp, scan_bytes, counts, offsets, (int)(len + 1), s);
    if (e != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    uint64_t total = 0;
    if ((e = hipMemcpyAsync(&total, offsets + len, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
        set_hip_error(e);
        return NQ_EDEVICE;
    }
    *out_len = total;
    if (!ocols || !old || !ord) return NQ_OK;                 // size query
    if (total > cap) return NQ_ERANGE;
    const uint64_t wgrid = (len + 63) / 64;
    if (wgrid > 0x7fffffffull) return NQ_EINVAL;
    hipLaunchKernelGGL(nq_expand_write_kernel, dim3((uint32_t)wgrid), dim3(64), 0, s, cols, ld,
                       rd, w, len, n, rows, offsets, ocols, old, ord, ow);
    if ((e = hipGetLastError()) != hipSuccess) { set_hip_error(e); return NQ_EDEVICE; }
    return NQ_OK;
}

}  // namespace nqi
