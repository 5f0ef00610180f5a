// zmc_family.hip -- one (integrand family, working precision) pair of scan
// kernels: compiled once per pair with -DZMC_FAMILY=<family template> and
// -DZMC_REAL=<float|double>, so the pairs build in parallel.
#include "zmc_tiles.hpp"

#if !defined(ZMC_FAMILY) || !defined(ZMC_REAL)
#error "zmc_family.hip needs -DZMC_FAMILY and -DZMC_REAL"
#endif

namespace zmc {
template struct FamilyOps<ZMC_FAMILY, ZMC_REAL>;
}  // namespace zmc
