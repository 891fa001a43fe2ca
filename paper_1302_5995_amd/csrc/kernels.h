// Launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace dtn {

// A pivot whose magnitude is at most this fraction of the largest entry of the
// block being factored marks the build as singular (DTN_ESINGULAR).
constexpr double kPivotRtol = 1e-11;

hipError_t launch_small(const SchurTask* tasks, int count, size_t lds, const int* ip, const DevBufs& B,
                        const Coef& C, DevStatus* st, hipStream_t s);
hipError_t launch_reset(const LargeMerge* lm, int nlm, const DevBufs& B, DevStatus* st, hipStream_t s);
hipError_t launch_large_gather(const LargeMerge* lm, int nlm, int blocks_per, const int* ip, const DevBufs& B,
                               const Coef& C, hipStream_t s);
hipError_t launch_gje_panel(int nt, int r, int w, const LargeMerge* lm, int nlm, int c0, int* ip, const DevBufs& B,
                            DevStatus* st, hipStream_t s);
hipError_t launch_gje_swap(const LargeMerge* lm, int nlm, int imax, int c0, const int* ip, const DevBufs& B,
                           hipStream_t s);
hipError_t launch_gje_kmap(const LargeMerge* lm, int nlm, int imax, int* ip, hipStream_t s);
hipError_t launch_gemm_batched(const GemmDesc* descs, int ndesc, int tiles, const DevBufs& B, const int* ip,
                               hipStream_t s);
hipError_t launch_gemm_single(const GemmDesc& D, const DevBufs& B, hipStream_t s);
hipError_t launch_scale_copy(const double* S, double* T, long long cnt, double scale, hipStream_t s);
hipError_t kernels_init();

}  // namespace dtn
