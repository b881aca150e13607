// Instantiates the specialised backward kernels for NI = DPD_NI (set on the
// compiler command line) and every L in 1..kSpecL.
#include "dpd_bwd_kernels.h"

#ifndef DPD_NI
#error "compile with -DDPD_NI=<1..8>"
#endif

#define DPD_CAT2(a, b) a##b
#define DPD_CAT(a, b) DPD_CAT2(a, b)

namespace dpd {

void DPD_CAT(register_bwd_ni, DPD_NI)(BwdTable &t)
{
    register_bwd_one<DPD_NI, 1>(t);
    register_bwd_one<DPD_NI, 2>(t);
    register_bwd_one<DPD_NI, 3>(t);
    register_bwd_one<DPD_NI, 4>(t);
    register_bwd_one<DPD_NI, 5>(t);
    register_bwd_one<DPD_NI, 6>(t);
    register_bwd_one<DPD_NI, 7>(t);
    register_bwd_one<DPD_NI, 8>(t);
}

}  // namespace dpd
