// placeholder until the block Jacobi SVD lands
#include "plan.h"
extern "C" dmrg_status dmrg_svd_truncate(dmrg_ctx_t, dmrg_basis_t, dmrg_basis_t, const int32_t*, const double*,
                                         int64_t, double, int64_t*, double*, int64_t, double*, int64_t,
                                         double*, int64_t, double*) {
  return dmrg::fail(DMRG_ENOTSUP, "svd: not built yet");
}
