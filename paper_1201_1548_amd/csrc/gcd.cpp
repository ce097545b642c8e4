#include "gcd.hpp"

namespace bires {

int gcd_bounds(const bires_upoly*, const bires_upoly*, int32_t*, int32_t*) { return BIRES_EINVAL; }
int run_gcd(Context*, const bires_upoly&, const bires_upoly&, bires_upoly*, int, hipStream_t) { return BIRES_EINVAL; }

}  // namespace bires
