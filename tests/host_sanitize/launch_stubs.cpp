// Host-only stand-ins for the kernel launchers of liblbm (lbm_internal.h),
// so that the host runtime (lbm_api.cpp) can be built with the host
// sanitizers and its argument checks, planning and error paths exercised
// without a GPU.  Every launcher reports that no device is present.
#include "lbm_internal.h"

namespace lbm {
hipError_t launch_rest_state(const Params&, const float*, float*, int*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_init_slots(const Params&, const Buffers&, int, int, int, bool, bool, hipStream_t, int, int) {
  return hipErrorNoDevice;
}
hipError_t launch_activate(const Params&, const Buffers&, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_fused(const Params&, const Buffers&, int, bool, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_criterion(const Params&, const Buffers&, int, int, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_inplace_psi(const Params&, const Buffers&, int, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_inplace_collide(const Params&, const Buffers&, int, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_candidates(const Params&, const Buffers&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_propose(const Params&, const Buffers&, int, int, int, const float*, float, float*, int32_t*, int,
                          hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_batch_offsets(const Batch&, const Params&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_batch_step(const Batch&, const Params&, int, bool, bool, bool, int, bool, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_export(const Params&, const Buffers&, int, int, float*, float*, float*, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_active_cells(const Params&, const Buffers&, uint8_t*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_repack(const Params&, const Buffers&, int, bool, hipStream_t) { return hipErrorNoDevice; }
hipError_t static_staging(float** out) {
  *out = nullptr;
  return hipErrorNoDevice;
}
hipError_t launch_mass(const Params&, const Buffers&, int, int, double*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_debug_fields(const Params&, const Buffers&, int, int, float*, float*, float*, hipStream_t) {
  return hipErrorNoDevice;
}
}  // namespace lbm
