/*
 * probe.h -- measurement probes that sit beside the engine (libflprobe.so).
 *
 * Not part of the method.  The complex64 sweep is bound by FP32 vector FMAs
 * (16 per amplitude and gate, Sec. III A's gate application written out as
 * real arithmetic), so its roofline needs the FMA rate the vector ALUs reach
 * without packed FP32 instructions.  On gfx950 that rate depends on the
 * operands: an FMA that reads a scalar register issues alone (one per cycle
 * per SIMD), while FMAs whose operands all sit in vector registers issue two
 * per cycle per SIMD when two waves have one ready.  These probes measure
 * both rates on the device.
 *
 * Errors: FL_OK (0), FL_EINVAL (-1) for a bad argument (nothing launched) or
 * FL_EHIP (-3) if the launch failed.
 */
#ifndef FLOQUET_PROBE_H
#define FLOQUET_PROBE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Enqueue one FMA-loop kernel on hip_stream (a hipStream_t, NULL = the
 * default stream): `blocks` workgroups of 256 threads, each thread running
 * `iters` rounds of 16 independent FP32 FMA chains x <- a x + b with a and b
 * in scalar registers, i.e.
 * 2 * 16 * iters * blocks * 256 flop.  out: caller-owned device buffer of
 * blocks * 256 floats (one result per thread, so nothing is optimised away).
 * blocks in [1, 2^20], iters in [1, 10^7]. */
int flp_fma_loop(float *out, int blocks, int iters, void *hip_stream);

/* The same loop (same arguments, recurrence and result) with both FMA
 * coefficients held in vector registers: the dual-issue rate. */
int flp_fma_loop_v(float *out, int blocks, int iters, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif
