// Host stand-ins for the kernel launchers of libseamcarve, for the sanitizer build of the C ABI's
// host code (argument validation, workspace layouts, the batch planner).  Every launch reports
// hipErrorNotSupported, so a call that gets past its validation returns SC_EHIP without touching
// device memory.  Test infrastructure only: built by tests/test_sanitize.py.
#include <hip/hip_runtime.h>

#include "sc_internal.h"

namespace sc {
namespace {
constexpr hipError_t kNo = hipErrorNotSupported;
}
hipError_t launch_energy_i32(const uint8_t*, int, int, int, long long, int32_t*, hipStream_t) { return kNo; }
hipError_t launch_prepare_single(const Img&, hipStream_t) { return kNo; }
hipError_t launch_prepare_from_i32(const Img&, const int32_t*, hipStream_t) { return kNo; }
hipError_t launch_carve_single(const Img&, int, int, int, hipStream_t) { return kNo; }
hipError_t launch_carve_steps(const Img*, int, int, int, unsigned long long, int*, const int4*, int, hipStream_t) {
    return kNo;
}
hipError_t launch_slot_write(Img*, int, const Img&, hipStream_t) { return kNo; }
hipError_t launch_unpack_dirs(const Img&, uint8_t*, hipStream_t) { return kNo; }
hipError_t launch_remove_seam(uint8_t*, int, int, int, long long, const int32_t*, hipStream_t) { return kNo; }
hipError_t launch_transpose(const uint8_t*, int, int, int, long long, uint8_t*, long long, hipStream_t) { return kNo; }
hipError_t launch_prepare_batch(const Img*, int, int, hipStream_t) { return kNo; }
hipError_t launch_carve_batch(const Img*, const int2*, const int2*, const int*, int, int, hipStream_t) { return kNo; }
// blocks of a variant per compute unit: the register-limited occupancy of the real kernels
int carve_blocks_per_cu(int v) { return 2048 / variant(v).threads; }
hipError_t launch_seam_origins(const int32_t*, int, int, int, int32_t*, int32_t*, hipStream_t) { return kNo; }
hipError_t launch_insert_seams(const uint8_t*, int, int, int, long long, int, const int32_t*, uint8_t*, long long,
                               hipStream_t) {
    return kNo;
}
hipError_t launch_obj_reset(ObjCtl*, int, hipStream_t) { return kNo; }
hipError_t launch_obj_carve(const ObjImg*, int, int, hipStream_t) { return kNo; }
hipError_t launch_mask_bbox(const uint8_t*, int, int, long long, int*, hipStream_t) { return kNo; }
hipError_t launch_copy_rows(const uint8_t*, long long, uint8_t*, long long, int, int, hipStream_t) { return kNo; }
hipError_t launch_fwt_prepare(const Img*, int, int, hipStream_t) { return kNo; }
hipError_t launch_fwt_carve(const Img*, const int2*, int, int, hipStream_t) { return kNo; }
int fwt_blocks_per_cu() { return 3; }
hipError_t noalloc_scratch(void**) { return kNo; }
hipError_t launch_copy_status(const unsigned*, uint32_t*, hipStream_t) { return kNo; }
}  // namespace sc
