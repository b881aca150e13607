// Instantiates the persistent batched kernel for S = DPD_BATCH_S samples per
// lane (set on the compiler command line; one object per S).
#include "dpd_batch_kernels.h"

#ifndef DPD_BATCH_S
#error "compile with -DDPD_BATCH_S=<2|4|8>"
#endif

#define DPD_CAT2(a, b) a##b
#define DPD_CAT(a, b) DPD_CAT2(a, b)

namespace dpd {

void DPD_CAT(register_batch_s, DPD_BATCH_S)(BatchTable &t)
{
    const int idx = DPD_BATCH_S == 2 ? 0 : (DPD_BATCH_S == 4 ? 1 : 2);
    t.fn[idx] = &launch_batch<DPD_BATCH_S>;
    t.kern[idx] = (const void *)&batch_kernel<DPD_BATCH_S>;
}

}  // namespace dpd
