// Binned push step: CSR_PUSH and SPARSE instantiations (see snp_step_bin.h).
#include "snp_step_bin.h"

namespace snp {

SNP_BIN_DEFINE_LAYOUT(L_CSR_PUSH)
SNP_BIN_DEFINE_LAYOUT(L_SPARSE)

}  // namespace snp
