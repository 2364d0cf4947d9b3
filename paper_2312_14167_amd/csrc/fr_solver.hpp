// Internal solver handle shared by the API layer and the kernel engines.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fr_host.hpp"

namespace frmi {

constexpr int WALL_CHUNK = 256;  // wall flux points per workgroup of the wall-force sum

// per-mesh free stream and viscosity in the state precision
template <typename T>
struct FlowDev {
  T rho, v[3], p, mu;
};

template <typename T, int P>
struct OpsDev {
  T D[P * P];   // D[a*P + b] = l_b'(xi_a)
  T lm[P], lp[P];
  T gp[P], gm[P];  // g_R'(xi_a), g_R'(-xi_a)
  // derivative with the interior part of the correction folded in:
  // Dt[a*P + b] = D[a*P + b] + g_R'(-xi_a) l_b(-1) - g_R'(xi_a) l_b(+1)
  T Dt[P * P];
};

// device operator tables in precision T (every entry rounded once from the FP64 host tables)
template <typename T, int P>
inline OpsDev<T, P> make_ops(const Ops1D &h) {
  OpsDev<T, P> o;
  for (int i = 0; i < P * P; ++i) o.D[i] = (T)h.D[i];
  for (int i = 0; i < P; ++i) {
    o.lm[i] = (T)h.lm[i];
    o.lp[i] = (T)h.lp[i];
    o.gp[i] = (T)h.gp[i];
    o.gm[i] = (T)h.gm[i];
  }
  for (int a = 0; a < P; ++a)
    for (int b = 0; b < P; ++b)
      o.Dt[a * P + b] = (T)(h.D[a * P + b] + h.gm[a] * h.lm[b] - h.gp[a] * h.lp[b]);
  return o;
}

template <typename T>
struct PhysDev {
  T gamma, gm1, prandtl, beta, tau;
  // side of an interior face pair that supplies the viscous part of the LDG common flux:
  // +1 (beta = 1/2: R), -1 (beta = -1/2: L), 0 (both sides, any other beta)
  int side;
};

// flux-point state u_f.  Where a face's NV x Nfp values (fb of `bytes` each) fill at least two
// 128-byte lines: element-major, then face, each face block (variable-major) padded to whole
// lines, and the stage kernels write only the faces read later, so every write covers whole
// lines.  Smaller faces: [Ne][NV][Nf] with every face written (skipping some would leave partly
// written lines, which cost more than the bytes they save).
constexpr bool uf_face_skip(int fb, int bytes) { return fb * bytes >= 256; }
// values per face block in the face-blocked layout
constexpr int uf_face_stride(int fb, int bytes) {
  return uf_face_skip(fb, bytes) ? (fb * bytes + 127) / 128 * 128 / bytes : fb;
}

// LDG flux side for beta in precision T
template <typename T>
inline int ldg_side_of(double beta) {
  const T b = (T)beta;
  return b == T(0.5) ? 1 : (b == T(-0.5) ? -1 : 0);
}

}  // namespace frmi

struct fr_solver {
  int dim = 0, p = 0, P = 0, Ns = 0, Nfp = 0, Nf = 0, NV = 0;
  int equations = 0, precision = 0;
  int64_t Ne = 0;
  int n_mesh = 1;
  size_t tsize = 8;
  double gamma = 1.4, prandtl = 0.71, beta = 0.5, tau = 0.1;

  // host copies
  frmi::Ops1D ops;
  std::vector<double> xsol;           // [Ne][Ns][dim]
  std::vector<double> h_rho, h_vel, h_p, h_mu;
  std::vector<int64_t> mesh_begin;
  std::vector<int64_t> h_wall_mesh_begin;
  std::vector<double> h_probe_pinf;

  // device arrays (precision T unless noted)
  void *metric = nullptr;   // [Ne][dim*dim+1][Ns]
  void *uf = nullptr;       // u_f: [Ne][2 dim][face stride] by face where faces fill two lines
                            // (uf_face_skip), else [Ne][NV][Nf]
  uint8_t *uf_faces = nullptr;  // [Ne] faces (bit f) whose u_f the stage kernels write
  void *fvn = nullptr;      // viscous normal flux at own flux points (NS), in the layout of uf
  void *vol = nullptr;      // [Ne][NV][Ns]   volume divergence (NS)
  void *fnrm = nullptr;     // [Ne][dim+1][Nf] outward unit normal at own flux points, then |N|
  void *fhat = nullptr;     // common flux x |N|, in the layout of uf
  void *acc = nullptr;      // [Ne][NV][Ns]
  void *ustage = nullptr;   // [Ne][NV][Ns]
  void *pair_nrm = nullptr; // [npair][dim+1]
  void *bnd_nrm = nullptr;  // [nbnd][dim+1]
  void *flow = nullptr;     // FlowDev<T>[n_mesh]
  int32_t *pairL = nullptr, *pairR = nullptr, *bnd = nullptr, *elem_mesh = nullptr;
  int32_t *nbr = nullptr;   // [Ne][Nf] neighbour code of every own flux point
  int64_t npair = 0, nbnd = 0, n_wall = 0;
  int64_t n_bc = 0;         // walls + far field; boundary points from n_bc on are mortar points
  void *ifc_uh = nullptr;   // [nbnd - n_bc][NV] common solution at mortar points (degree groups)
  double *bnd_w = nullptr;          // FP64 [nbnd]
  int64_t *wall_mesh_begin = nullptr;  // device [n_mesh+1]

  // probes and accumulators (FP64)
  int n_probe = 0, cap = 0, forces = 0;
  int64_t *probe_elem = nullptr;  // [n_probe]
  double *probe_w = nullptr;      // [n_probe][Ns]
  double *probe_pinf = nullptr;   // [n_probe]
  double *probe_coef = nullptr;   // [n_probe][NV + dim] probe adjoint coefficients (scratch)
  double *series = nullptr;       // [n_probe][cap]
  double *sums = nullptr;         // [n_probe][2]
  double *force_acc = nullptr;    // [n_mesh][dim]
  int wall_nchunk = 0;            // wall-force partial sums per mesh (chunks of WALL_CHUNK points)
  double *wall_partial = nullptr; // [n_mesh][wall_nchunk][dim]
  unsigned long long *count = nullptr;  // [0] samples taken, [1] probe workgroups done in the
                                        // current sample (k_probe's ticket)
  int *nonfinite = nullptr;

  // time stepping / graphs
  int64_t steps_since_reset = 0;
  hipStream_t cap_stream = nullptr;
  // reverse segments of the trajectory adjoint captured as graphs, keyed by their arguments
  struct SegGraph {
    hipGraphExec_t ex = nullptr;
    const void *states = nullptr, *stages = nullptr, *res = nullptr, *pbar = nullptr, *ubar = nullptr;
    const double *dt = nullptr;
    double *xbar = nullptr;
    int n = 0;
  };
  std::vector<SegGraph> seg_graphs;
  hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};  // (sample, fresh u_f) variants
  void *graph_u[4] = {nullptr, nullptr, nullptr, nullptr};
  const double *graph_dt[4] = {nullptr, nullptr, nullptr, nullptr};
  int use_graphs = 1;
  // autotuner choice per volume kernel (0: default tile, 1: half, 2: quarter)
  // autotuner candidate per kernel kind: NS volume, NS lifting + RK, Euler volume + RK, NS volume
  // adjoint
  int tune[4] = {0, 0, 0, 0};

  // per-kernel event timing (FR_K_* ids)
  int profiling = 0;
  struct ProfRec { int id; hipEvent_t a, b; };
  mutable std::vector<ProfRec> prof_pending;
  mutable std::vector<hipEvent_t> prof_pool;
  double prof_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t prof_n[8] = {0, 0, 0, 0, 0, 0, 0, 0};

  // mesh-node adjoint: host copy of the mesh; tables and work arrays uploaded / allocated on first use
  int device = 0;  // HIP device current at fr_build_operators (all device arrays live there)
  int geom_q = 1;
  int64_t n_node = 0;
  std::vector<double> h_node_xyz;
  std::vector<int64_t> h_elem_nodes;
  int geo_nn = 0;
  double *geo_Xe = nullptr;       // [Ne][nn][dim] element node coordinates
  double *geo_dphi_s = nullptr;   // [dim][Ns][nn]
  double *geo_dphi_f = nullptr;   // [dim][Nf][nn]
  double *geo_Xeb = nullptr;      // [Ne][nn][dim] per-element node adjoint
  int32_t *geo_inc_ptr = nullptr, *geo_inc = nullptr;
  void *geo_Gm = nullptr;         // [Ne][dim*dim+1][Ns] adjoint of S rows and 1/J (state precision)
  void *geo_Gn = nullptr;         // [Ne][dim+1][Nf] adjoint of the unit normal and |N| at own flux points
  void *geo_R = nullptr;          // [Ne][nv][Ns] forward residual at the linearisation state
  int geo_deferred = 0;           // between fr_geo_adjoint_begin / _end: accumulate, map once
  double *probe_dw = nullptr;     // [n_probe][dim][Ns] d weights / d xi
  double *probe_dxi = nullptr;    // [n_probe][nn][dim][dim] d xi_k / d X_{n,j}
  int64_t *probe_nodes = nullptr; // [n_probe][nn]

  // VJP work arrays (allocated on first use)
  void *vjp_work = nullptr;
  size_t vjp_bytes = 0;
  char *adj_work = nullptr;  // RK-step adjoint: 7 state-sized arrays

  std::vector<void *> owned;  // everything hipMalloc'ed
};
