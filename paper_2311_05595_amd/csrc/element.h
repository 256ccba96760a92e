// Host-side element matrices of Lagrange and serendipity rectangular-prism
// elements.
#pragma once

#include <vector>

namespace mgcg {

// The n^3 sub-element stiffness matrices K^(e_i) of one unit displacement
// element of the given order (1: 8 nodes, 2: 27 nodes, 3: 64 nodes) with
// modulus 1 and Poisson ratio nu, as [n^3][nd][nd] row-major,
// nd = 3 * (order+1)^3.  Sub-element i = sx + n*(sy + n*sz); local node
// a = ax + (p+1)*(ay + (p+1)*az); local DOF 3a + c.
// family 0: Lagrange; 1: serendipity of degree 2 or 3 (its 20 or 32 nodes
// in the Lagrange layout of that degree, zero rows and columns elsewhere)
std::vector<double> sub_element_matrices(int order, int nsub, double nu, int family = 0);

// Trilinear weight of coarse vertex b (bits x,y,z of b in {0,1}) at the
// node with coarse-local lattice position (px,py,pz) in {0..r}^3 (spacing
// 1/r of the coarse element).
double trilinear_weight(int px, int py, int pz, int b, int r = 2);

}  // namespace mgcg
