// residual_gather.hip -- the fused from-mesh kernel (mesh_kernel.hpp) with u
// given per vertex, [n_vert][N_comp], and a P1 coefficient given per vertex,
// [n_vert][N_coef], both gathered through the connectivity; coefficients at
// the points or per cell stay per element.
#include "mesh_kernel.hpp"

namespace femq {

hipError_t launch_residual_gather(int dim, int phys, int rule, int space, int dtype, const MeshArgs& a,
                                  const Launch& l) {
    const MeshDispatch<true> f{dtype, a, l};
    return dispatch_element(dim, phys, rule, space, f, hipErrorInvalidValue);
}

}  // namespace femq
