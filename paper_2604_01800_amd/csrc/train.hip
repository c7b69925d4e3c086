// Training of the DeepONet (Eq. 19 residual loss, Adam).
#include <hip/hip_runtime.h>

#include "api_internal.hpp"
#include "net_internal.hpp"

namespace ppe {

struct TrainState {};

void net_train_free(ppe_net* n) {
  delete n->train;
  n->train = nullptr;
}

}  // namespace ppe
