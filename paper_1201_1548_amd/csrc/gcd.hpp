// Modular gcd in Z[x] (Brown's method, Section 5.1 "Computing gcds in Z[x]").
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/bires.h"
#include "engine.hpp"

namespace bires {

int gcd_bounds(const bires_upoly* a, const bires_upoly* b, int32_t* max_degree, int32_t* max_limbs);
int run_gcd(Context* cx, const bires_upoly& a, const bires_upoly& b, bires_upoly* out, int mem, hipStream_t st);

}  // namespace bires
