// Modular gcd in Z[x] (Brown's method, Section 5.1 "Computing gcds in Z[x]").
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/bires.h"
#include "engine.hpp"

namespace bires {

int gcd_bounds(const bires_upoly* a, const bires_upoly* b, int32_t* max_degree, int32_t* max_limbs);
int run_gcd(Context* cx, const bires_upoly& a, const bires_upoly& b, bires_upoly* out, int mem, hipStream_t st);
int run_squarefree(Context* cx, const bires_upoly& r, bires_upoly* unit, bires_upoly* factors, int32_t max_factors,
                   int32_t* count, int mem, hipStream_t st);

}  // namespace bires
