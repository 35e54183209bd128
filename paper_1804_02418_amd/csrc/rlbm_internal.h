// Internal declarations of the rlbm library (not part of the C ABI).
#pragma once

#include <cstddef>
#include <cstdint>
#include <cstdio>

#include "rlbm_math.h"

namespace rlbm {

struct Quadrature {
    double w1[4], w2[4], p0[4];
};

// Polished quadrature and force matrices (computed once, host only).
// Returns false with *err set when the set-up self-checks fail.
bool host_constants(Quadrature *q, double Cx[kK][kK], double Cy[kK][kK], const char **err);

// Largest violation of the third-order conditions (all monomials of degree
// <= 6, each divided by max(|moment|, 1)) by a massless quadrature on the
// 48-node stencil; quadrature_search.cpp.
double massless_stencil_residual(const Quadrature &q);

}  // namespace rlbm
