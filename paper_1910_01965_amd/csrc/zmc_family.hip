// zmc_family.hip -- the scan kernels of one integrand family in one working
// precision for eight integration dimensions: compiled once per triple with
// -DZMC_FAMILY=<family template>, -DZMC_REAL=<float|double> and
// -DZMC_NLO=<1|9> (N = 1..8 or 9..16), so the triples build in parallel.
#include "zmc_tiles.hpp"

#if !defined(ZMC_FAMILY) || !defined(ZMC_REAL) || !defined(ZMC_NLO)
#error "zmc_family.hip needs -DZMC_FAMILY, -DZMC_REAL and -DZMC_NLO"
#endif

namespace zmc {
template struct FamilyOps<ZMC_FAMILY, ZMC_REAL, ZMC_NLO>;
}  // namespace zmc
