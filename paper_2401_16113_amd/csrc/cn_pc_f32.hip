// float instantiation of the preconditioner transform kernels.
#include "cn_pc_kernels.hpp"

namespace cn {

#define CN_FWD_CASE_f32(L) \
  case L:                 \
    return fwd_cand<float, L>(cand, Lc, it, j, v, pitch, s);
#define CN_INV_CASE_f32(L) \
  case L:                 \
    return inv_cand<float, L>(cand, Lc, it, j, z, zf, pitch, s);
#define CN_INFO_CASE_f32(L) \
  case L:                  \
    return cand_info<float, L>(ci, B, T, S, FS);

CN_DEFINE_PC_PRECISION(float, f32)

}  // namespace cn
