/*
 * hlbm_reference.h -- a bandwidth reference beside the HLBM sweep (part of
 * libhlbm.so, not of the method).
 *
 * The fused stream-collide sweep of the homogenized lattice BGK scheme moves,
 * per cell and step, 19 pulled populations in, 19 populations out and one
 * porosity value in (Sec. 3.2: the collision is cell-local, so streaming is
 * the whole of the data movement).  hlbm_ref_stream_pattern performs exactly
 * those loads and stores -- the pull g*_i(x) = g_i(x - c_i) of the D3Q19 FP32
 * populations of a fully periodic box, with the sweep's own gather, row pitch,
 * block geometry and non-temporal stores, plus the read of the FP32 porosity
 * value -- and leaves the collision out.  Timed beside the sweep, it shows how
 * much of the sweep's time the access pattern itself sets.
 */
#ifndef HLBM_REFERENCE_H
#define HLBM_REFERENCE_H

#ifdef __cplusplus
extern "C" {
#endif

/* One pull-streaming pass: dst row i, cell x = src row i, cell x - c_i
 * (periodic wrap), for the 19 D3Q19 populations; the porosity value of each
 * cell is read and folded in as 0 * d (the written values are the pulled ones
 * for finite d).
 *   src, dst: device buffers of 19 FP32 rows, row i starting at element
 *             i * P, P = nx*ny*nz + row_pad_bytes / 4 (the population row
 *             pitch of hlbm_config::row_pad_bytes); they must not overlap.
 *   d:        device array of nx*ny*nz FP32 values.
 *   block_x:  threads per block along x (multiple of 64, <= 1024).
 *   stream:   hipStream_t, NULL = default stream.
 * Enqueues one kernel and returns 0, or -1 (HLBM_EINVAL) for a bad argument
 * (NULL pointer, a size outside [1, 1024] per axis, row_pad_bytes not a
 * multiple of 4, block_x out of range), or -3 (HLBM_EDEVICE) if the launch
 * fails. */
int hlbm_ref_stream_pattern(const void *src, void *dst, const void *d, int nx, int ny, int nz,
                            int row_pad_bytes, int block_x, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HLBM_REFERENCE_H */
