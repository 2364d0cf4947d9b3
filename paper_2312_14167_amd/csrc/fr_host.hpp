// Host-side construction of the FR operators, curved-element metrics, face connectivity and
// probe tables.  Plain C++17 (no HIP types); results are uploaded by the API layer.
#pragma once
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace frmi {

// element flux-point neighbour code: >= 0 -> partner (element * Nf + flux point), bit 30 set when
// this element is the R side of the pair; < 0 -> boundary point -(code + 1)
constexpr int32_t NBR_R_BIT = 1 << 30;

// Internal face tag of a degree-group solver: a face whose partner has another solution degree.
// Its flux points are boundary points after the walls and the far field; their common solution
// comes from a buffer and their common flux from the mortar kernels of the whole mesh.
constexpr int32_t BC_MORTAR = 3;

// Thrown by host construction; mapped to an fr_status at the ABI.
struct FrError : std::runtime_error {
  int code;
  FrError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// 1-D operators on P = p+1 Gauss-Legendre points (all FP64).
struct Ops1D {
  int P = 0;
  std::vector<double> xi, w;   // nodes, weights
  std::vector<double> D;       // D[a*P + b] = l_b'(xi_a)
  std::vector<double> lm, lp;  // l_b(-1), l_b(+1)
  std::vector<double> gp, gm;  // g_R'(xi_a), g_R'(-xi_a) for the g_DG correction function
};

Ops1D build_ops_1d(int p);

// Gauss-Lobatto-Legendre nodes of degree q (q+1 points, q in 1..4).
std::vector<double> gll_nodes(int q);

struct MeshIn {
  int dim = 0, p = 0, q = 0;
  int64_t n_elem = 0, n_node = 0;
  const double *node_xyz = nullptr;
  const int64_t *elem_nodes = nullptr;
  const int32_t *face_bc = nullptr;
  int n_periodic = 0;
  const double *periodic_vec = nullptr;
  int n_mesh = 1;
  std::vector<int64_t> mesh_begin;  // n_mesh + 1
  bool allow_mortar = false;        // degree-group solver: BC_MORTAR faces allowed
};

struct Geometry {
  int dim = 0, P = 0, Ns = 0, Nfp = 0, Nf = 0;
  int64_t n_elem = 0;
  std::vector<double> metric;  // [Ne][dim*dim + 1][Ns]: S[k][j] (k*dim + j), then 1/J
  std::vector<double> J;       // [Ne][Ns]
  std::vector<double> xsol;    // [Ne][Ns][dim]
  std::vector<double> xf;      // [Ne][Nf][dim]
  std::vector<double> Nvec;    // [Ne][Nf][dim] scaled outward normal s_f S[k_f, :]
};

Geometry build_geometry(const MeshIn &m, const Ops1D &ops);

struct Connectivity {
  // interior / periodic flux-point pairs, sorted by the L code; code = e * Nf + fpt
  std::vector<int32_t> pairL, pairR;
  std::vector<double> pair_nrm;   // [npair][dim + 1]: unit normal of the L side, |N|
  // boundary flux points: walls first [0, n_wall), then far field
  std::vector<int32_t> bnd;
  std::vector<double> bnd_nrm;    // [nbnd][dim + 1]
  std::vector<double> bnd_w;      // face quadrature weight of the flux point (walls: force integral)
  int64_t n_wall = 0;
  int64_t n_bc = 0;               // walls + far field; mortar points follow
  std::vector<int64_t> wall_mesh_begin;  // [n_mesh + 1] ranges into the wall list
  std::vector<int32_t> elem_mesh;        // [Ne]
  // per element flux point: partner code (bit 30 set on the R side) or -(boundary index + 1)
  std::vector<int32_t> nbr;              // [Ne][Nf]
  // [Ne][dim + 1][Nf] outward unit normal (R side: -n_L exactly), then |N| of the face pair (the L
  // side's, on both sides) or of the boundary point
  std::vector<double> fnrm;
};

Connectivity build_connectivity(const MeshIn &m, const Ops1D &ops, const Geometry &g);

struct Probe {
  int64_t elem = -1;
  int mesh = 0;
  std::vector<double> xi;       // reference coordinates
  std::vector<double> weights;  // [Ns] tensor Lagrange weights
  // derivatives for the mesh-node adjoint (the probe is fixed in physical space, so its
  // reference coordinates move with the element's nodes: d xi / d X_n = -A^{-1} phi_n(xi))
  std::vector<double> dweights;  // [dim][Ns] d weights / d xi_k
  std::vector<double> dxi;       // [nn][dim][dim]: [n][j][k] = d xi_k / d X_{n,j}
  std::vector<int64_t> nodes;    // [nn] global ids of the element's nodes
};

Probe locate_probe(const MeshIn &m, const Ops1D &ops, const double *xp, int mesh);

// reference coordinates [Nf][dim] of the flux points of degree o.P - 1: face f on coordinate f/2 at
// side -1 (f even) / +1 (f odd), tangential Gauss points lowest coordinate fastest
std::vector<double> ref_flux_points(int dim, const Ops1D &o);

// physical coordinates [n][dim] of reference points ref [n][dim] in element e
std::vector<double> map_ref_points(const MeshIn &m, int64_t e, const std::vector<double> &ref);

// Tables of the mesh-node adjoint: element node coordinates, derivatives of the geometry basis
// at solution and flux points, and the node -> (element, local node) incidence in a fixed order.
struct GeoAdj {
  int nn = 0;
  std::vector<double> Xe;        // [Ne][nn][dim]
  std::vector<double> dphi_s;    // [dim][Ns][nn]
  std::vector<double> dphi_f;    // [dim][Nf][nn]
  std::vector<int32_t> inc_ptr;  // [n_node + 1]
  std::vector<int32_t> inc;      // element * nn + local node, grouped by node, increasing
};

GeoAdj build_geo_adj(const MeshIn &m, const Ops1D &ops);

}  // namespace frmi
