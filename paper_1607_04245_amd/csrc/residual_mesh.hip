// residual_mesh.hip -- the fused from-mesh kernel (mesh_kernel.hpp) with u
// and the coefficient given per element (closure rows).
#include "mesh_kernel.hpp"

namespace femq {

hipError_t launch_residual_mesh(int dim, int phys, int rule, int space, int dtype, const MeshArgs& a,
                                const Launch& l) {
    const MeshDispatch<false> f{dtype, a, l};
    return dispatch_element(dim, phys, rule, space, f, hipErrorInvalidValue);
}

}  // namespace femq
