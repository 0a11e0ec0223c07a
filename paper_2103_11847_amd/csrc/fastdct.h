// Tube transforms in O(p log p) per tube for power-of-two tube lengths.
#pragma once
#include "internal.h"

namespace dctk {

constexpr int kFastMinTube = 16;  // shortest tube of the fast transform (a workgroup holds at most 256 tubes)

// Longest tube of the fast transform for DCTK_F32 / DCTK_F64 (one workgroup holds a whole tube in LDS).
int tube_fast_max(int dtype);
// p is a power of two within [kFastMinTube, tube_fast_max(dtype)].
bool tube_fast_shape_ok(int dtype, int64_t p);
// out = in x_3 G, G = matrix `which` (DCTK_MAT_*) of transform `tube`, in O(p log p) per tube; dtype
// DCTK_F32 or DCTK_F64 for both buffers; enqueued on s, allocates nothing.
hipError_t launch_tube_fast(dctk_ctx ctx, hipStream_t s, int tube, int which, int dtype, int64_t p, int64_t count,
                            const void* in, void* out);
// The same transform as a step of a c-product (operators with tubes longer than
// kMaxTube): scale = true for the input side (L, L^{-T}: the control block's
// input scale s, xnorm (may be null) receives s * in, out may be a 16-bit GEMM
// type), epi = true for the output side (L^{-1}, L^T: out = a * (in x_3 G) +
// b * src, per-workgroup partials of out^2 in ctl.part_out, their number in
// *nblocks_out).  Batchable (recorded while planning).
hipError_t launch_tube_fast_ctl(dctk_ctx ctx, hipStream_t s, int tube, int which, int in_dtype, int out_dtype,
                                int64_t p, int64_t count, const void* in, void* out, const void* src, void* xnorm,
                                const Ctl& ctl, bool scale, bool epi, int* nblocks_out);

}  // namespace dctk
