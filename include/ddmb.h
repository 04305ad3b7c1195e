/*
 * ddmb.h -- C ABI of the microbenchmark library libddmb.so (gfx950).
 *
 * Measures the rates that bound the dedispersion kernels on the machine itself,
 * as denominators for their roofline fractions: the VALU issue rate of each
 * integer add form the accumulate loops use, the LDS read bandwidth per access
 * width and alignment (the shared-memory bandwidth that the analysis of Sec. 5.1
 * prices per accumulated sample), and the HBM copy bandwidth.
 *
 * Every launch function enqueues one kernel on `stream` (a hipStream_t passed as
 * void*, NULL = default stream) and returns a hipError_t value (0 = success,
 * hipErrorInvalidValue for a bad argument, nothing enqueued then).  The caller
 * times the launch (HIP events) and divides the counted work by the time.  All
 * pointers are device memory the caller owns; nothing is allocated.
 */
#ifndef DDMB_H
#define DDMB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* VALU instruction forms: 0 v_add_u32, 1 v_add3_u32, 2 v_pk_add_u16,
 * 3 v_add_u32 with an SDWA high-half operand, 4 v_perm_b32, 5 the 8-bit
 * accumulate pair (two v_perm_b32 and two v_add3_u32 per 8 sample-adds).
 * ddmb_valu_instructions_per_lane: instructions each lane issues in one launch.
 * ddmb_valu: `blocks` workgroups of 256 lanes; d_in holds 128 uint32 operands,
 * d_out receives blocks * 256 uint32 (one per lane, so nothing is dead code). */
int ddmb_valu_instructions_per_lane(int form, int iters);
int ddmb_valu(int form, int blocks, int iters, const void *d_in, void *d_out, void *stream);

/* LDS reads of `width` (4, 8 or 16) bytes per lane, lane-contiguous, starting
 * `misalign` (0..15) bytes past a 16-byte boundary; `blocks` workgroups of 256
 * lanes, each holding 48 KiB of LDS; d_out receives blocks * 256 uint32.
 * ddmb_lds_bytes_per_lane: bytes each lane reads in one launch. */
int ddmb_lds_bytes_per_lane(int width, int iters);
int ddmb_lds(int width, int misalign, int blocks, int iters, void *d_out, void *stream);

/* Copy `bytes` (a multiple of 16) from d_src to d_dst, both 16-byte aligned,
 * with `blocks` workgroups of 256 lanes (16 bytes per lane per step). */
int ddmb_copy(const void *d_src, void *d_dst, size_t bytes, int blocks, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DDMB_H */
