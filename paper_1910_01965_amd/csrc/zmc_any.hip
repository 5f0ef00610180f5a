// zmc_any.hip -- the any-family batch kernel of one working precision,
// compiled once per precision with -DZMC_REAL=<float|double>.
#include "zmc_tiles.hpp"

#if !defined(ZMC_REAL)
#error "zmc_any.hip needs -DZMC_REAL"
#endif

namespace zmc {
template struct AnyOps<ZMC_REAL>;
}  // namespace zmc
