// Definition of the opaque plan / batch objects and host helpers shared by
// the host translation units of libdpd.
#pragma once

#include <mutex>
#include <vector>

#include "dpd.h"
#include "dpd_internal.h"

struct dpd_plan {
    int device = 0;
    dpd::CoefMap map;
    int32_t K = 0;
    dpd_tune tune;
    std::vector<float> raw;      // host copy of the 2K coefficient floats
    float *d_table = nullptr;    // precombined table (device)
    float *d_table_call = nullptr;  // table of the calls that pass device coefficients
                                    // (same allocation as d_table, right after it)
    float *h_stage = nullptr;    // pinned staging of dpd_set_coeffs_async (created on first use)
    hipEvent_t staged = nullptr; // recorded after the last copy out of h_stage
    int8_t ls_slot[32] = {};     // least squares: LDS row slot of each basis entry,
    std::once_flag ls_once;      // chosen on the first least-squares call
};

namespace dpd {

dpd_status hip_fail(hipError_t e);
dpd_status make_map(const int32_t *mo, int32_t nm, const int32_t *co, int32_t nc, int32_t L,
                    CoefMap &map);
hipError_t launch_prep(const CoefMap &map, const void *raw, float *M, hipStream_t stream,
                       const int32_t *flag = nullptr);
dpd_status run_forward(const CoefMap &map, const dpd_tune &tune, const float *M, hipStream_t stream,
                       const void *in, void *out, int64_t rows, int64_t n, int64_t ld,
                       const void *hist);
dpd_status check_io(const void *in, const void *out, int64_t rows, int64_t n, int64_t ld);
dpd_tune default_tune();
bool valid_tune(const dpd_tune &t);
void ls_layout(const CoefMap &map, int8_t *slot);

}  // namespace dpd
