// placeholder, replaced by the MFMA separable kernel
#include "dev_common.h"
namespace e2e {
hipError_t launch_sep_mfma(const FrameDev *, const KernelCfg &, const int2 *, int, int *, int *,
                           hipStream_t)
{
    return hipErrorNotSupported;
}
}  // namespace e2e
