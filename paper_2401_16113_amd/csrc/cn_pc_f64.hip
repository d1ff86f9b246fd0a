// double instantiation of the preconditioner transform kernels.
#include "cn_pc_kernels.hpp"

namespace cn {

#define CN_FWD_CASE_f64(L) \
  case L:                 \
    return fwd_cand<double, L>(cand, Lc, it, j, v, pitch, s);
#define CN_INV_CASE_f64(L) \
  case L:                 \
    return inv_cand<double, L>(cand, Lc, it, j, z, zf, pitch, s);
#define CN_INFO_CASE_f64(L) \
  case L:                  \
    return cand_info<double, L>(ci, B, T, S, FS);

CN_DEFINE_PC_PRECISION(double, f64)

}  // namespace cn
