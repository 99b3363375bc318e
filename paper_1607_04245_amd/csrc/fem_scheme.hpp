// fem_scheme.hpp -- the compile-time "scheme" of an element kernel, which
// packs the quadrature rule and the coefficient space into one template
// argument, and the dispatcher that maps runtime (dim, physics, rule, space)
// to kernel template instances.
#pragma once

#include <hip/hip_runtime.h>

#include "fem.h"

namespace femq {

__host__ __device__ constexpr int scheme(int rule, int space) { return rule | (space << 2); }
__host__ __device__ constexpr int rule_of(int s) { return s & 3; }
__host__ __device__ constexpr int space_of(int s) { return s >> 2; }

// F provides `template <int DIM, int PHYS, int SCHEME> R operator()()`.
template <int D, int P, int RU, typename F, typename R>
static R dispatch_space(int space, const F& f, R bad) {
    switch (space) {
    case FEM_COEF_QUAD: return f.template operator()<D, P, scheme(RU, FEM_COEF_QUAD)>();
    case FEM_COEF_P1: return f.template operator()<D, P, scheme(RU, FEM_COEF_P1)>();
    case FEM_COEF_P0: return f.template operator()<D, P, scheme(RU, FEM_COEF_P0)>();
    default: return bad;
    }
}

template <int D, int P, typename F, typename R>
static R dispatch_rule(int rule, int space, const F& f, R bad) {
    if (rule == FEM_RULE_CENTROID) return dispatch_space<D, P, FEM_RULE_CENTROID>(space, f, bad);
    if constexpr (D == 2) {
        if (rule == FEM_RULE_TRI3) return dispatch_space<D, P, FEM_RULE_TRI3>(space, f, bad);
    } else {
        if (rule == FEM_RULE_TET4) return dispatch_space<D, P, FEM_RULE_TET4>(space, f, bad);
    }
    return bad;
}

template <int D, typename F, typename R>
static R dispatch_phys(int phys, int rule, int space, const F& f, R bad) {
    switch (phys) {
    case FEM_LAPLACE: return dispatch_rule<D, FEM_LAPLACE>(rule, space, f, bad);
    case FEM_ELASTICITY: return dispatch_rule<D, FEM_ELASTICITY>(rule, space, f, bad);
    case FEM_MASS: return dispatch_rule<D, FEM_MASS>(rule, space, f, bad);
    default: return bad;
    }
}

template <typename F, typename R>
static R dispatch_element(int dim, int phys, int rule, int space, const F& f, R bad) {
    if (dim == 2) return dispatch_phys<2>(phys, rule, space, f, bad);
    if (dim == 3) return dispatch_phys<3>(phys, rule, space, f, bad);
    return bad;
}

}  // namespace femq
