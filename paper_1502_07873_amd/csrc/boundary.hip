// Absorbing edges: the first-order Clayton-Engquist relation on the left,
// right and bottom edges (the paper's condition on the artificial boundary,
// discretised with the centred time difference of Section 3.3.1).
//
// At an edge node with outward normal n and tangent t the relation is
//   u_t = -(1/rho) (n n^T / c_p + t t^T / c_s) sigma(u) n.
// Written out with the normal derivative one-sided into the grid, the
// tangential one central (one-sided at the ends of the edge), and the node's
// own same-component term at the mean of levels m+1 and m-1, every component
// w of an edge node takes the form
//   w^{m+1} = ((1 - a) w^{m-1} + 2 (a w_in + b T)) / (1 + a)
// with w_in the same component on the neighbour one node inside, T a
// tangential difference (times h) of the other component, a = c dt / h for
// the wave speed of that component's direction and b = a or
// lambda dt / (rho c_p h):
//   left   (i = 0):    u: a_p, u_{1},     + l Dz v      v: a_s, v_{1},     + a_s Dz u
//   right  (i = nx-1): u: a_p, u_{nx-2},  - l Dz v      v: a_s, v_{nx-2},  - a_s Dz u
//   bottom (k = nz-1): u: a_s, u_{nz-2},  - a_s Dx v    v: a_p, v_{nz-2},  - l Dx u
// (Dz w = (w_{k+1} - w_{k-1}) / 2, or the one-sided difference at the top and
// bottom of a side column; Dx likewise along the bottom row.)  Corners take
// their column's relation.  The interior kernels never write edge nodes, so
// this kernel and the interior step of the same level are independent.  The
// one-step kernels marked `edges` in the variant table run the same node
// updates (ce.h) in extra wavefronts of their own launch instead.
#include "ce.h"
#include "internal.h"

namespace eig {

namespace {

// One block per running solve; threads stride over its edge nodes.
__global__ void __launch_bounds__(256) ce_edge_kernel(const SolveDesc* __restrict__ descs,
                                                      int step) {
    const SolveDesc& d = descs[blockIdx.x];
    const int m = step - d.start;
    if (m < 0 || m >= d.nsteps) return;
    const int nb = 2 * d.nz + d.nx - 2;
    for (int e = threadIdx.x; e < nb; e += blockDim.x) ce_edge_node(d, m, e);
}

}  // namespace

void launch_ce_edges(const SolveDesc* descs, int n, int step, hipStream_t s) {
    if (n > 0) ce_edge_kernel<<<n, 256, 0, s>>>(descs, step);
}

}  // namespace eig
