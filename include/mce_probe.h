/*
 * mce_probe.h -- C ABI of libmce_probe.so, the peak-rate microbenchmarks
 * that give the roofline denominators of the search kernel on the device at
 * hand (a measurement aid beside libmce.so, not an operation of the paper).
 *
 * Both run on the current HIP device and the default stream, allocate and
 * free their own small buffers, and wait for their kernel.  Return 0, -1 for
 * a bad argument (NULL output, zero blocks or iterations), -4 for a HIP error.
 */
#ifndef MCE_PROBE_H
#define MCE_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 32-bit integer vector ALU rate: `blocks` workgroups of 256 lanes, each lane
 * running 16 independent chains of `iters` x (XOR, AND, OR) one-instruction
 * operations.  *lane_ops_per_s = lane-operations per second (one wave64
 * instruction = 64 of them); *seconds (may be NULL) = the kernel's time. */
int mce_probe_valu(uint32_t blocks, uint32_t iters, double *lane_ops_per_s, double *seconds);

/* LDS read rate: `blocks` workgroups of 256 lanes, each lane reading four
 * 16-byte words of a 16 KB LDS buffer per iteration, consecutive lanes on
 * consecutive words (no bank conflicts).  *bytes_per_s = bytes read per
 * second; *seconds (may be NULL) = the kernel's time. */
int mce_probe_lds(uint32_t blocks, uint32_t iters, double *bytes_per_s, double *seconds);

#ifdef __cplusplus
}
#endif

#endif /* MCE_PROBE_H */
