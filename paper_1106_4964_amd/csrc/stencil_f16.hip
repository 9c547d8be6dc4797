// Stencil kernels at F16 storage (instantiated for 18- and 12-real links).
#include "stencil_kernels.h"

namespace ovl {

void launch_stencil_f16(const StencilArgs& A, int recon, int nrhs, Shape sh, hipStream_t s) {
  if (recon == 18)
    launch_pr<OVL_F16, 18>(A, nrhs, sh, s);
  else
    launch_pr<OVL_F16, 12>(A, nrhs, sh, s);
}

}  // namespace ovl
