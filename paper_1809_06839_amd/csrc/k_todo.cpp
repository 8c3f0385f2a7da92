// Launchers not yet implemented report hipErrorNotSupported (mapped to
// MIAUG_EDEVICE by the ABI layer).
#include "internal.h"
namespace miaug {
hipError_t launch_c2(const uint8_t *, int, int, int, const float *, const int32_t *, int, int, uint8_t *, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_wc_fwd(const float *, int, int, int, int, const float *, float *, hipStream_t) { return hipErrorNotSupported; }
size_t wc_workspace_bytes(int, int, int, int) { return 0; }
hipError_t launch_wc_bwd(const float *, int, int, int, int, const float *, const float *, float *, float *, void *,
                         hipStream_t) { return hipErrorNotSupported; }
size_t elastic_workspace_bytes(int, int, int) { return 0; }
hipError_t launch_elastic_fields(uint64_t, uint64_t, int, int, int, double, int, int, int32_t *, void *, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_grid_tables(const double *, int, int, int, int32_t *, int32_t *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_elastic_grid_u8(const uint8_t *, const uint8_t *, int, int, int, int, const int32_t *, const int32_t *,
                                  const int32_t *, uint8_t *, uint8_t *, int, hipStream_t) { return hipErrorNotSupported; }
size_t chain_f32_workspace_bytes(int, int, int, int) { return 0; }
hipError_t launch_chain_f32_fwd(const float *, int, int, int, int, const int32_t *, const int32_t *, const int32_t *,
                                float *, void *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_chain_f32_bwd(const float *, int, int, int, int, const int32_t *, const int32_t *, const int32_t *,
                                float *, void *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_image_stats(const uint8_t *, int, int64_t, int, uint64_t *, int32_t *, int32_t *, uint32_t *,
                              hipStream_t) { return hipErrorNotSupported; }
}  // namespace miaug
