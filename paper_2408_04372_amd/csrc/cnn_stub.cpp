// Learned preconditioning stage: placeholder until the CNN kernels are built.
#include "handle.hpp"

namespace stmg {
struct CnnState {};
void cnn_free(CnnState* c) { delete c; }
stmg_status cnn_precondition(stmg_handle*, const double*, double*, double*, bool* used) {
  *used = false;
  return STMG_OK;
}
}  // namespace stmg
