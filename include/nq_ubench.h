/*
 * libnq microbenchmarks -- the measurements behind the DFS kernel's roofline
 * (measurement code, not part of the counting path).
 *
 * The paper's kernel is limited by the core's integer issue rate and by its
 * per-thread stack in shared memory, whose layout it makes bank-conflict-free
 * (Section 3.1).  These two calls measure the same two resources on the
 * current GPU.  Both return NQ_OK or a negative NQ_E* status (include/nq.h);
 * NQ_EINVAL for arguments outside the stated ranges, NQ_EDEVICE for a HIP
 * failure (nq_last_hip_error()).  Both allocate and free their own small
 * device buffers and are synchronous on the null stream.
 */
#ifndef NQ_UBENCH_H_
#define NQ_UBENCH_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * nq_ubench_valu -- int32 VALU issue rate of one operation.
 *
 * Launches 4 * waves_per_simd single-wave workgroups per CU (waves_per_simd
 * in [1, 8]); every lane runs `chains` (1 or 8) independent dependency chains
 * of `iters` operations each (iters > 0, a multiple of 8) of op: 0 = v_add3_u32,
 * 1 = v_bitop3_b32, 2 = v_cndmask_b32 with an SGPR lane mask, 3 = v_addc_co_u32
 * with an SGPR carry-in, 4 = v_add_lshl_u32, 5 = v_xad_u32, 6 = v_and_b32,
 * 7 = v_xor_b32, 8 = v_or3_b32, 9 = v_sub_u32, 10 = v_lshrrev_b32,
 * 11 = v_add_u32.  *kernel_ms = the
 * launch's event time; *mean_cycles = the shader-clock cycles (s_memtime) a
 * wave spent in its loop, averaged over the waves.  Lane-operations executed =
 * CUs * 4 * waves_per_simd * 64 * chains * iters.
 */
int nq_ubench_valu(uint32_t op, uint32_t chains, uint32_t waves_per_simd, uint64_t iters,
                   double* kernel_ms, double* mean_cycles);

/*
 * nq_ubench_lds -- the DFS stack's LDS accesses.
 *
 * Launches waves_per_cu single-wave workgroups per CU (1..32, within the LDS
 * of a CU), each with frames * 1 KiB of LDS (frames in [2, 32]) holding a
 * 16-byte frame per lane and level.  The first active_lanes (1..64) lanes of
 * every wave repeat `iters` times, at levels that differ across the lanes of
 * a wave: op 0 = write one frame at the current level (ds_write_b128) and read
 * the frame of the next level (ds_read_b128); 1 = the read only; 2 = the
 * write only; 3 = one 16-byte exchange at the current level
 * (ds_wrxchg2_rtn_b64 of two adjacent qwords: writes a frame and returns the
 * one it replaces); 4 = as 0 with 8-byte accesses (b64); 5 = as 0 with 4-byte
 * accesses (b32); 6 = write b64 only; 7 = write b32 only; 8 = write b96 only;
 * 9 = write 16 bytes as ds_write2_b64 (two adjacent qwords) only; 10 = read
 * b96 only; 11 = read 16 bytes as ds_read2_b64 only; 12 = as 0 with 12-byte
 * accesses (b96) in the same 16-byte slots; each iteration waits for its
 * accesses.  layout 0 =
 * lane-interleaved (frame f of lane l at byte (f * 64 + l) * 16, the DFS
 * kernel's stack), 1 = per-lane contiguous (lane l's frames at
 * (l * frames + f) * 16).  *kernel_ms = the launch's event time.  LDS
 * instructions = CUs * waves_per_cu * iters * (2 for ops 0, 4, 5, 12; 1 else).
 * op in [0, 12].
 */
int nq_ubench_lds(uint32_t layout, uint32_t op, uint32_t active_lanes, uint32_t waves_per_cu,
                  uint32_t frames, uint64_t iters, double* kernel_ms);

#ifdef __cplusplus
}
#endif

#endif /* NQ_UBENCH_H_ */
