#include "dpd_plan.h"
#define DPD_EXPORT extern "C" __attribute__((visibility("default")))
DPD_EXPORT dpd_status dpd_batch_create(const dpd_stream_desc *d, int32_t, const dpd_tune *, dpd_batch **o) { return (!d || !o) ? DPD_EINVAL : DPD_EUNSUPPORTED; }
DPD_EXPORT dpd_status dpd_batch_apply(dpd_batch *, void *) { return DPD_EUNSUPPORTED; }
DPD_EXPORT dpd_status dpd_batch_apply_each(dpd_batch *, void *) { return DPD_EUNSUPPORTED; }
DPD_EXPORT dpd_status dpd_batch_info(const dpd_batch *, int64_t *, int32_t *) { return DPD_EUNSUPPORTED; }
DPD_EXPORT dpd_status dpd_batch_destroy(dpd_batch *b) { return b ? DPD_EUNSUPPORTED : DPD_OK; }
