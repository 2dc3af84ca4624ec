// Binned push step: OPTIMIZED (Sy) and SLICED instantiations (see snp_step_bin.h).
#include "snp_step_bin.h"

namespace snp {

SNP_BIN_DEFINE_LAYOUT(L_OPT)
SNP_BIN_DEFINE_LAYOUT(L_SLICED)

}  // namespace snp
