// placeholder replaced by the product implementation
#include "hmat_internal.h"
namespace hm {
hmat_status multiply(HMat*, HMat*, double, const Opts&, HMat**) {
  throw Error(HMAT_ERR_INTERNAL, "multiply not built yet");
}
hmat_status multiply_batched(HMat* const*, HMat* const*, int32_t, double, const Opts&, HMat**, int32_t*) {
  throw Error(HMAT_ERR_INTERNAL, "multiply not built yet");
}
}
