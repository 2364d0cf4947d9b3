// Flux reconstruction with a solution degree per element: the sponge of the airfoil case's
// computational details, where the degree falls from 4 (or 3) near the airfoil to 0 towards the
// outer boundaries so that acoustic waves are damped before they reach them.
//
// Every degree group is a solver of its own over its elements (same kernels as a one-degree mesh;
// degree 0 is one point per element with correction derivative 1/2).  A face between two degrees
// p_lo < p_hi is a boundary face of both groups ("mortar points", after the walls and the far
// field in each group's boundary list) and is coupled on the higher side's flux points:
//   k_mortar_sol:  the lower side's trace polynomial (through its own face points, tensor
//                  Lagrange basis I) at the mortar points; the LDG common solution there goes to
//                  the higher side's mortar points, its L2 projection onto the lower face
//                  (Pi = W_lo^-1 I^T W_m, Gauss quadrature on the mortar points) to the lower
//                  side's;
//   k_mortar_flux: Rusanov flux along the L side's normal, each side's own viscous normal flux
//                  carried to the mortar (the lower side's through I), LDG weights and penalty,
//                  x |N| of the higher side -> the higher side's transformed common flux, its
//                  projection (negated) -> the lower side's, so both sides integrate the same
//                  flux over the face and the scheme stays conservative.
// One RK stage: mortar solution, every group's volume / common-flux kernel, mortar flux, every
// group's lifting + RK kernel.  The whole step is captured once into a HIP graph and replayed.
// The state is one buffer: the groups in increasing degree, each [n_elem][NV][Ns] with its
// elements in increasing element number, each group starting on a 64-value boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fr.h"
#include "fr_device.hpp"
#include "fr_dispatch.hpp"

using namespace frmi;

namespace {

constexpr int MAX_GROUPS = 5;         // degrees 0..4
constexpr int MORTAR_BS = 64;         // one workgroup (one wave) per mortar face
constexpr int MAX_MORTAR_PTS = 25;    // (p_hi + 1)^(dim - 1)
constexpr int MAX_LO_PTS = 16;        // (p_lo + 1)^(dim - 1), p_lo < p_hi
constexpr int64_t STATE_ALIGN = 64;   // values: group states start on 256-byte boundaries

#define VD_HIP_OK(expr)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw FrError(e_ == hipErrorOutOfMemory ? FR_ERR_OOM : FR_ERR_HIP,                     \
                    std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

// one degree group's arrays as the mortar kernels see them
template <typename T>
struct GroupDev {
  const T *uf;        // own flux-point states (the degree's u_f layout)
  const T *fvn;       // own viscous normal flux (u_f layout)
  T *fhat;            // transformed common normal flux (u_f layout)
  T *ifc_uh;          // [mortar point][NV] common solution at the mortar points
  const T *bnd_nrm;   // [boundary point][dim + 1] outward unit normal, |N|
  int64_t n_bc;       // walls + far field: mortar point q is boundary point n_bc + q
  int P, Nfp, Nf;
  int skip, EB, FST, VS;  // u_f layout: face-blocked (skip) or [Ne][NV][Nf]; strides
};

struct MortarFace {
  int32_t g_hi, g_lo;  // degree groups of the higher / lower side
  int32_t e_hi, e_lo;  // element inside its group
  int32_t f_hi, f_lo;  // face of the element
  int32_t q_hi, q_lo;  // mortar-point index of the face's first point in each group
  int32_t tab;         // offset of the face's tables: I [Nm][Nlo], then Pi [Nlo][Nm]
  int32_t hi_is_L;     // the higher side is the L side (L: the smaller (element, face))
  int8_t perm[16];     // lower-degree canonical point j -> the lower face's flux point
};

template <typename T>
__device__ __forceinline__ int64_t gpt(const GroupDev<T> &g, int64_t e, int fp) {
  return g.skip ? e * g.EB + (int64_t)(fp / g.Nfp) * g.FST + fp % g.Nfp : e * g.EB + fp;
}

// the lower side's u_f and (lo_f != nullptr) its viscous normal flux at its face points, in
// canonical order, into LDS: the workgroup loads each value once, one per lane
template <int D, typename T>
__device__ __forceinline__ void stage_lower(const MortarFace &mf, const int8_t *perm, const GroupDev<T> &L,
                                            T (*lo_u)[D + 2], T (*lo_f)[D + 2]) {
  constexpr int NV = D + 2;
  const int Nlo = L.Nfp;
  for (int k = (int)threadIdx.x; k < Nlo * NV; k += MORTAR_BS) {
    const int v = k / Nlo, j = k % Nlo;
    const int fp = mf.f_lo * Nlo + perm[j];
    lo_u[j][v] = L.uf[gpt(L, mf.e_lo, fp) + v * L.VS];
    if (lo_f) lo_f[j][v] = L.fvn[gpt(L, mf.e_lo, fp) + v * L.VS];
  }
}

// at mortar point i: the higher side's own value of variable-major array `ah` (u_f layout) and the
// lower side's trace polynomial there, from its staged face values lo
template <int D, typename T>
__device__ __forceinline__ void mortar_pair(const MortarFace &mf, const GroupDev<T> &H, const T *ah,
                                            const T (*lo)[D + 2], int Nlo, const T *I, int i, T *vh, T *vl) {
  constexpr int NV = D + 2;
  const int Nm = H.Nfp;
  const int64_t ph = gpt(H, mf.e_hi, mf.f_hi * Nm + i);
  for (int v = 0; v < NV; ++v) {
    vh[v] = ah[ph + v * H.VS];
    vl[v] = T(0);
  }
  for (int j = 0; j < Nlo; ++j) {
    const T c = I[i * Nlo + j];
    for (int v = 0; v < NV; ++v) vl[v] += c * lo[j][v];
  }
}

// LDG common solution u^ = (1/2 + beta) u_L + (1/2 - beta) u_R at the mortar points and its
// projection onto the lower face
template <int D, typename T>
__global__ __launch_bounds__(MORTAR_BS) void k_mortar_sol(const MortarFace *__restrict__ faces,
                                                          const GroupDev<T> *__restrict__ grp,
                                                          const T *__restrict__ tabs, T wl, T wr) {
  constexpr int NV = D + 2;
  __shared__ T lu[MAX_MORTAR_PTS][NV];
  __shared__ T llo[MAX_LO_PTS][NV];
  const MortarFace mf = faces[blockIdx.x];
  const int8_t *perm = faces[blockIdx.x].perm;
  const GroupDev<T> H = grp[mf.g_hi], L = grp[mf.g_lo];
  const int Nm = H.Nfp, Nlo = L.Nfp;
  const T *I = tabs + mf.tab, *Pi = I + Nm * Nlo;
  const int i = threadIdx.x;
  stage_lower<D, T>(mf, perm, L, llo, nullptr);
  __syncthreads();
  if (i < Nm) {
    T uh[NV], ul[NV];
    mortar_pair<D, T>(mf, H, H.uf, llo, Nlo, I, i, uh, ul);
    for (int v = 0; v < NV; ++v) {
      const T w = mf.hi_is_L ? wl * uh[v] + wr * ul[v] : wl * ul[v] + wr * uh[v];
      lu[i][v] = w;
      H.ifc_uh[(int64_t)(mf.q_hi + i) * NV + v] = w;
    }
  }
  __syncthreads();
  if (i < Nlo) {
    T s[NV];
    for (int v = 0; v < NV; ++v) s[v] = T(0);
    for (int m = 0; m < Nm; ++m) {
      const T c = Pi[i * Nm + m];
      for (int v = 0; v < NV; ++v) s[v] += c * lu[m][v];
    }
    for (int v = 0; v < NV; ++v) L.ifc_uh[(int64_t)(mf.q_lo + perm[i]) * NV + v] = s[v];
  }
}

// common normal flux at the mortar points, along n_L, x |N|:
// Rusanov(u_L, u_R) - [(1/2 - beta) f_L - (1/2 + beta) f_R - tau (u_L - u_R)], f_X each side's
// viscous flux along its own outward normal; the higher side takes it with its sign, the lower
// side its projection with the opposite sign
template <int D, typename T>
__global__ __launch_bounds__(MORTAR_BS) void k_mortar_flux(const MortarFace *__restrict__ faces,
                                                           const GroupDev<T> *__restrict__ grp,
                                                           const T *__restrict__ tabs, PhysDev<T> ph) {
  constexpr int NV = D + 2;
  __shared__ T lf[MAX_MORTAR_PTS][NV];
  __shared__ T llo[MAX_LO_PTS][NV], llf[MAX_LO_PTS][NV];
  const MortarFace mf = faces[blockIdx.x];
  const int8_t *perm = faces[blockIdx.x].perm;
  const GroupDev<T> H = grp[mf.g_hi], L = grp[mf.g_lo];
  const int Nm = H.Nfp, Nlo = L.Nfp;
  const T *I = tabs + mf.tab, *Pi = I + Nm * Nlo;
  const T sh = mf.hi_is_L ? T(1) : T(-1);
  const int i = threadIdx.x;
  stage_lower<D, T>(mf, perm, L, llo, llf);
  __syncthreads();
  if (i < Nm) {
    T uh[NV], ul[NV], fh[NV], fl[NV];
    mortar_pair<D, T>(mf, H, H.uf, llo, Nlo, I, i, uh, ul);
    {
      const int fph = mf.f_hi * Nm + i;
      for (int v = 0; v < NV; ++v) {
        fh[v] = H.fvn[gpt(H, mf.e_hi, fph) + v * H.VS];
        fl[v] = T(0);
      }
      for (int j = 0; j < Nlo; ++j) {
        const T c = I[i * Nlo + j];
        for (int v = 0; v < NV; ++v) fl[v] += c * llf[j][v];
      }
    }
    const T *bn = H.bnd_nrm + (H.n_bc + mf.q_hi + i) * (D + 1);
    T n[D];
    for (int j = 0; j < D; ++j) n[j] = sh * bn[j];  // n_L
    const T mag = bn[D];
    T uL[NV], uR[NV], fL[NV], fR[NV];
    for (int v = 0; v < NV; ++v) {
      uL[v] = mf.hi_is_L ? uh[v] : ul[v];
      uR[v] = mf.hi_is_L ? ul[v] : uh[v];
      fL[v] = mf.hi_is_L ? fh[v] : fl[v];
      fR[v] = mf.hi_is_L ? fl[v] : fh[v];
    }
    T F[NV];
    rusanov<D>(uL, uR, n, ph.gamma, ph.gm1, F);
    const T wlf = T(0.5) - ph.beta, wrf = T(0.5) + ph.beta;
    const int64_t po = gpt(H, mf.e_hi, mf.f_hi * Nm + i);
    for (int v = 0; v < NV; ++v) {
      const T Fm = (F[v] - (wlf * fL[v] - wrf * fR[v] - ph.tau * (uL[v] - uR[v]))) * mag;
      lf[i][v] = Fm;
      H.fhat[po + v * H.VS] = sh * Fm;
    }
  }
  __syncthreads();
  if (i < Nlo) {
    T s[NV];
    for (int v = 0; v < NV; ++v) s[v] = T(0);
    for (int m = 0; m < Nm; ++m) {
      const T c = Pi[i * Nm + m];
      for (int v = 0; v < NV; ++v) s[v] += c * lf[m][v];
    }
    const int64_t po = gpt(L, mf.e_lo, mf.f_lo * Nlo + perm[i]);
    for (int v = 0; v < NV; ++v) L.fhat[po + v * L.VS] = -sh * s[v];
  }
}

double lagrange(const std::vector<double> &x, int b, double t) {
  double v = 1.0;
  for (size_t m = 0; m < x.size(); ++m)
    if ((int)m != b) v *= (t - x[m]) / (x[b] - x[m]);
  return v;
}

}  // namespace

struct fr_vdeg {
  int dim = 0, NV = 0, precision = 0, tsize = 0, n_group = 0, device = 0;
  int deg[MAX_GROUPS] = {};
  fr_solver *child[MAX_GROUPS] = {};
  Dispatch dsp[MAX_GROUPS] = {};
  int64_t n_elem[MAX_GROUPS] = {}, offset[MAX_GROUPS + 1] = {};
  std::vector<int64_t> elems[MAX_GROUPS];  // global element ids of each group, increasing
  int64_t n_mortar = 0;
  MortarFace *faces = nullptr;
  void *grp = nullptr, *tabs = nullptr;
  double gamma = 1.4, prandtl = 0.71, beta = 0.5, tau = 0.1;
  int n_probe = 0, forces = 0;
  std::vector<int> probe_group, probe_slot;
  std::vector<void *> owned;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph[4] = {};
  void *graph_u[4] = {};
  const double *graph_dt[4] = {};
  int64_t steps_since_reset = 0;
  int use_graphs = 1;
};

namespace {

void vd_destroy(fr_vdeg *v) {
  if (!v) return;
  for (int k = 0; k < 4; ++k)
    if (v->graph[k]) (void)hipGraphExecDestroy(v->graph[k]);
  for (int g = 0; g < MAX_GROUPS; ++g)
    if (v->child[g]) fr_destroy(v->child[g]);
  for (void *p : v->owned) (void)hipFree(p);
  if (v->cap_stream) (void)hipStreamDestroy(v->cap_stream);
  delete v;
}

template <typename X>
void *vd_upload(fr_vdeg *v, const std::vector<X> &h) {
  void *d = nullptr;
  const size_t bytes = std::max<size_t>(8, h.size() * sizeof(X));
  if (hipMalloc(&d, bytes) != hipSuccess) {
    (void)hipGetLastError();
    throw FrError(FR_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  v->owned.push_back(d);
  if (!h.empty()) VD_HIP_OK(hipMemcpy(d, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice));
  return d;
}

template <typename T>
void upload_groups(fr_vdeg *v, const std::vector<double> &tab) {
  std::vector<GroupDev<T>> gd(v->n_group);
  for (int g = 0; g < v->n_group; ++g) {
    const fr_solver *c = v->child[g];
    GroupDev<T> &d = gd[g];
    d.uf = (const T *)c->uf;
    d.fvn = (const T *)c->fvn;
    d.fhat = (T *)c->fhat;
    d.ifc_uh = (T *)c->ifc_uh;
    d.bnd_nrm = (const T *)c->bnd_nrm;
    d.n_bc = c->n_bc;
    d.P = c->P;
    d.Nfp = c->Nfp;
    d.Nf = c->Nf;
    const int fb = c->NV * c->Nfp;
    d.skip = uf_face_skip(fb, (int)sizeof(T)) ? 1 : 0;
    const int fs = uf_face_stride(fb, (int)sizeof(T));
    d.EB = 2 * c->dim * fs;
    d.FST = d.skip ? fs : c->Nfp;
    d.VS = d.skip ? c->Nfp : c->Nf;
  }
  v->grp = vd_upload(v, gd);
  std::vector<T> t(tab.begin(), tab.end());
  v->tabs = vd_upload(v, t);
}

template <int D, typename T>
void launch_mortar(const fr_vdeg *v, int phase, hipStream_t st) {
  PhysDev<T> ph;
  ph.gamma = (T)v->gamma;
  ph.gm1 = (T)(v->gamma - 1.0);
  ph.prandtl = (T)v->prandtl;
  ph.beta = (T)v->beta;
  ph.tau = (T)v->tau;
  ph.side = 0;
  const dim3 grid((unsigned)v->n_mortar);
  if (phase == 0)
    k_mortar_sol<D, T><<<grid, MORTAR_BS, 0, st>>>(v->faces, (const GroupDev<T> *)v->grp, (const T *)v->tabs,
                                                   T(0.5) + ph.beta, T(0.5) - ph.beta);
  else
    k_mortar_flux<D, T><<<grid, MORTAR_BS, 0, st>>>(v->faces, (const GroupDev<T> *)v->grp, (const T *)v->tabs, ph);
}

void mortar(const fr_vdeg *v, int phase, hipStream_t st) {
  if (v->n_mortar == 0) return;
  if (v->dim == 2)
    v->precision == FR_FP64 ? launch_mortar<2, double>(v, phase, st) : launch_mortar<2, float>(v, phase, st);
  else
    v->precision == FR_FP64 ? launch_mortar<3, double>(v, phase, st) : launch_mortar<3, float>(v, phase, st);
}

char *group_state(const fr_vdeg *v, const void *u, int g) {
  return (char *)u + v->offset[g] * v->tsize;
}

// one classical RK4 step of the whole mesh (see fr_rk_step)
void vd_step(const fr_vdeg *v, void *u, const double *dt, bool sample, bool fresh, hipStream_t st) {
  if (sample)
    for (int g = 0; g < v->n_group; ++g) v->dsp[g].sample_probes(v->child[g], group_state(v, u, g), st);
  if (fresh)
    for (int g = 0; g < v->n_group; ++g) v->dsp[g].interp(v->child[g], group_state(v, u, g), st);
  for (int k = 0; k < 4; ++k) {
    mortar(v, 0, st);
    for (int g = 0; g < v->n_group; ++g) v->dsp[g].stage_k(v->child[g], group_state(v, u, g), dt, k, sample, 1, st);
    mortar(v, 1, st);
    for (int g = 0; g < v->n_group; ++g) v->dsp[g].stage_k(v->child[g], group_state(v, u, g), dt, k, sample, 2, st);
  }
}

void vd_rhs(const fr_vdeg *v, const void *u, void *r, hipStream_t st) {
  for (int g = 0; g < v->n_group; ++g) v->dsp[g].interp(v->child[g], group_state(v, u, g), st);
  mortar(v, 0, st);
  for (int g = 0; g < v->n_group; ++g)
    v->dsp[g].rhs_part(v->child[g], group_state(v, u, g), group_state(v, r, g), 1, st);
  mortar(v, 1, st);
  for (int g = 0; g < v->n_group; ++g)
    v->dsp[g].rhs_part(v->child[g], group_state(v, u, g), group_state(v, r, g), 2, st);
}

fr_status vd_fail(int code, const std::string &msg) { return set_error(code, msg); }

}  // namespace

extern "C" {

fr_status fr_vdeg_build(const fr_mesh_desc *mesh, const int32_t *elem_degree, const fr_params *prm, fr_vdeg **out) {
  if (!out) return vd_fail(FR_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!mesh || !prm || !elem_degree) return vd_fail(FR_ERR_ARG, "mesh, degrees or params is NULL");
  if (mesh->dim != 2 && mesh->dim != 3) return vd_fail(FR_ERR_ARG, "dim must be 2 or 3");
  if (mesh->n_elem <= 0 || mesh->n_node <= 0 || !mesh->node_xyz || !mesh->elem_nodes || !mesh->face_bc)
    return vd_fail(FR_ERR_ARG, "empty mesh or NULL mesh array");
  if (mesh->geom_q < 1 || mesh->geom_q > 4) return vd_fail(FR_ERR_UNSUPPORTED, "geom_q must be in 1..4");
  if (mesh->n_periodic < 0 || (mesh->n_periodic > 0 && !mesh->periodic_vec))
    return vd_fail(FR_ERR_ARG, "bad periodic vectors");
  if (mesh->n_mesh > 1) return vd_fail(FR_ERR_UNSUPPORTED, "a variable-degree solver takes one mesh");
  if (prm->equations != FR_NAVIER_STOKES)
    return vd_fail(FR_ERR_UNSUPPORTED, "variable degree is built for the Navier-Stokes equations only");
  if (prm->precision != FR_FP64 && prm->precision != FR_FP32) return vd_fail(FR_ERR_ARG, "bad precision");
  if (prm->n_probe < 0 || (prm->n_probe > 0 && (!prm->probe_xyz || prm->max_samples <= 0)))
    return vd_fail(FR_ERR_ARG, "bad probe arguments");
  if (prm->probe_mesh)
    for (int a = 0; a < prm->n_probe; ++a)
      if (prm->probe_mesh[a] != 0) return vd_fail(FR_ERR_ARG, "probe mesh out of range");
  const int d = mesh->dim, nface = 2 * d, NV = d + 2;
  const int64_t Ne = mesh->n_elem;
  for (int64_t e = 0; e < Ne; ++e)
    if (elem_degree[e] < 0 || elem_degree[e] > 4) return vd_fail(FR_ERR_ARG, "element degree outside 0..4");
  fr_vdeg *v = new (std::nothrow) fr_vdeg();
  if (!v) return vd_fail(FR_ERR_OOM, "host allocation failed");
  try {
    v->dim = d;
    v->NV = NV;
    v->precision = prm->precision;
    v->tsize = prm->precision == FR_FP64 ? 8 : 4;
    v->gamma = prm->gamma;
    v->prandtl = prm->prandtl;
    v->beta = prm->ldg_beta;
    v->tau = prm->ldg_tau;
    v->forces = prm->forces ? 1 : 0;
    int nn = 1;
    for (int k = 0; k < d; ++k) nn *= mesh->geom_q + 1;
    // face partners of the whole mesh from its degree-0 connectivity (one flux point per face)
    MeshIn mf;
    mf.dim = d;
    mf.p = 0;
    mf.q = mesh->geom_q;
    mf.n_elem = Ne;
    mf.n_node = mesh->n_node;
    mf.node_xyz = mesh->node_xyz;
    mf.elem_nodes = mesh->elem_nodes;
    mf.face_bc = mesh->face_bc;
    mf.n_periodic = mesh->n_periodic;
    mf.periodic_vec = mesh->periodic_vec;
    mf.n_mesh = 1;
    mf.mesh_begin = {0, Ne};
    const Ops1D o0 = build_ops_1d(0);
    Connectivity c0;
    std::vector<double> fcent;  // [Ne][nface][d] face centres
    {
      Geometry g0 = build_geometry(mf, o0);
      c0 = build_connectivity(mf, o0, g0);
      fcent = std::move(g0.xf);
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t n = 0; n < mesh->n_node; ++n)
      for (int j = 0; j < d; ++j) {
        lo[j] = std::min(lo[j], mesh->node_xyz[n * d + j]);
        hi[j] = std::max(hi[j], mesh->node_xyz[n * d + j]);
      }
    double scale = 0.0;
    for (int j = 0; j < d; ++j) scale = std::max(scale, hi[j] - lo[j]);
    // groups: increasing degree, elements increasing
    std::vector<int> gidx(Ne, -1);
    std::vector<int64_t> lidx(Ne, -1);
    for (int p = 0; p <= 4; ++p) {
      std::vector<int64_t> el;
      for (int64_t e = 0; e < Ne; ++e)
        if (elem_degree[e] == p) el.push_back(e);
      if (el.empty()) continue;
      const int g = v->n_group++;
      v->deg[g] = p;
      v->n_elem[g] = (int64_t)el.size();
      for (size_t k = 0; k < el.size(); ++k) {
        gidx[el[k]] = g;
        lidx[el[k]] = (int64_t)k;
      }
      v->elems[g] = std::move(el);
    }
    auto partner = [&](int64_t e, int f, int64_t &e2, int &f2) {
      const int32_t code = c0.nbr[(size_t)e * nface + f];
      if (code < 0) return false;
      const int32_t c = code & (NBR_R_BIT - 1);
      e2 = c / nface;
      f2 = c % nface;
      return true;
    };
    // face tags of the groups: faces to another degree become mortar faces
    std::vector<int32_t> tag(mesh->face_bc, mesh->face_bc + Ne * nface);
    for (int64_t e = 0; e < Ne; ++e)
      for (int f = 0; f < nface; ++f) {
        int64_t e2;
        int f2;
        if (partner(e, f, e2, f2) && elem_degree[e2] != elem_degree[e]) tag[(size_t)e * nface + f] = BC_MORTAR;
      }
    // mortar-point index of every mortar face's first point inside its group (the order of the
    // group's boundary list: element, face, point)
    std::vector<int32_t> q0((size_t)Ne * nface, -1);
    for (int g = 0; g < v->n_group; ++g) {
      const int P = v->deg[g] + 1, Nfp = d == 2 ? P : P * P;
      int64_t q = 0;
      for (int64_t e : v->elems[g])
        for (int f = 0; f < nface; ++f)
          if (tag[(size_t)e * nface + f] == BC_MORTAR) {
            q0[(size_t)e * nface + f] = (int32_t)q;
            q += Nfp;
          }
      if (q >= ((int64_t)1 << 31) / NV) throw FrError(FR_ERR_ARG, "too many mortar points");
    }
    // probes: the lowest-index element containing the point decides the group
    v->n_probe = prm->n_probe;
    std::vector<std::vector<double>> gprobe(MAX_GROUPS);
    for (int a = 0; a < prm->n_probe; ++a) {
      const Probe pr = locate_probe(mf, o0, prm->probe_xyz + (size_t)a * d, 0);
      const int g = gidx[pr.elem];
      v->probe_group.push_back(g);
      v->probe_slot.push_back((int)(gprobe[g].size() / d));
      gprobe[g].insert(gprobe[g].end(), prm->probe_xyz + (size_t)a * d, prm->probe_xyz + (size_t)(a + 1) * d);
    }
    // mortar faces (listed from the higher side) and their I / Pi tables per
    // (higher degree, lower degree, face direction of the higher side)
    std::vector<MortarFace> faces;
    std::vector<double> tab;
    std::map<std::tuple<int, int, int>, int32_t> tab_of;
    std::vector<Ops1D> ops(5);
    for (int p = 0; p <= 4; ++p) ops[p] = build_ops_1d(p);
    for (int64_t e = 0; e < Ne; ++e)
      for (int f = 0; f < nface; ++f) {
        int64_t e2;
        int f2;
        if (!partner(e, f, e2, f2) || elem_degree[e] <= elem_degree[e2]) continue;
        const int ph = elem_degree[e], pl = elem_degree[e2];
        const int PH = ph + 1, PL = pl + 1;
        const int Nm = d == 2 ? PH : PH * PH, Nlo = d == 2 ? PL : PL * PL;
        const int k = f / 2;
        int others[2], no = 0;
        for (int m = 0; m < d; ++m)
          if (m != k) others[no++] = m;
        MortarFace M{};
        M.g_hi = gidx[e];
        M.g_lo = gidx[e2];
        M.e_hi = (int32_t)lidx[e];
        M.e_lo = (int32_t)lidx[e2];
        M.f_hi = f;
        M.f_lo = f2;
        M.q_hi = q0[(size_t)e * nface + f];
        M.q_lo = q0[(size_t)e2 * nface + f2];
        M.hi_is_L = (e < e2 || (e == e2 && f < f2)) ? 1 : 0;
        // canonical lower-degree points: the lower degree's Gauss points along the higher face's
        // tangential coordinates (lowest coordinate fastest), mapped through the higher element,
        // translated onto the lower face (periodic faces) and matched to its flux points
        std::vector<double> can((size_t)Nlo * d), rl((size_t)Nlo * d);
        for (int j = 0; j < Nlo; ++j) {
          const int t[2] = {j % PL, j / PL};
          can[(size_t)j * d + k] = (f % 2) ? 1.0 : -1.0;
          for (int a = 0; a < d - 1; ++a) can[(size_t)j * d + others[a]] = ops[pl].xi[t[a]];
        }
        const std::vector<double> rf = ref_flux_points(d, ops[pl]);
        std::copy(rf.begin() + (size_t)f2 * Nlo * d, rf.begin() + (size_t)(f2 + 1) * Nlo * d, rl.begin());
        const std::vector<double> xc = map_ref_points(mf, e, can), xl = map_ref_points(mf, e2, rl);
        double shl[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < d; ++j)
          shl[j] = fcent[((size_t)e2 * nface + f2) * d + j] - fcent[((size_t)e * nface + f) * d + j];
        std::vector<int> used(Nlo, 0);
        for (int j = 0; j < Nlo; ++j) {
          int best = -1;
          double bd = 1e300;
          for (int t = 0; t < Nlo; ++t) {
            double dist = 0.0;
            for (int c = 0; c < d; ++c) {
              const double dx = xc[(size_t)j * d + c] + shl[c] - xl[(size_t)t * d + c];
              dist += dx * dx;
            }
            if (dist < bd) {
              bd = dist;
              best = t;
            }
          }
          if (std::sqrt(bd) > 1e-7 * scale || used[best])
            throw FrError(FR_ERR_MESH, "non-conforming face between degrees at element " + std::to_string(e));
          used[best] = 1;
          M.perm[j] = (int8_t)best;
        }
        const auto key = std::make_tuple(ph, pl, k);
        auto it = tab_of.find(key);
        if (it == tab_of.end()) {
          const int32_t off = (int32_t)tab.size();
          const std::vector<double> rh = ref_flux_points(d, ops[ph]);
          std::vector<double> I((size_t)Nm * Nlo), Pi((size_t)Nlo * Nm);
          for (int i = 0; i < Nm; ++i)
            for (int j = 0; j < Nlo; ++j) {
              const int t[2] = {j % PL, j / PL};
              double val = 1.0;
              for (int a = 0; a < d - 1; ++a)
                val *= lagrange(ops[pl].xi, t[a], rh[((size_t)(2 * k) * Nm + i) * d + others[a]]);
              I[(size_t)i * Nlo + j] = val;
            }
          for (int j = 0; j < Nlo; ++j) {
            const double wl = ops[pl].w[j % PL] * (d == 3 ? ops[pl].w[j / PL] : 1.0);
            for (int i = 0; i < Nm; ++i) {
              const double wm = ops[ph].w[i % PH] * (d == 3 ? ops[ph].w[i / PH] : 1.0);
              Pi[(size_t)j * Nm + i] = I[(size_t)i * Nlo + j] * wm / wl;
            }
          }
          tab.insert(tab.end(), I.begin(), I.end());
          tab.insert(tab.end(), Pi.begin(), Pi.end());
          it = tab_of.emplace(key, off).first;
        }
        M.tab = it->second;
        faces.push_back(M);
      }
    // the degree groups (device work starts here)
    for (int g = 0; g < v->n_group; ++g) {
      std::vector<int64_t> en((size_t)v->n_elem[g] * nn);
      std::vector<int32_t> fb((size_t)v->n_elem[g] * nface);
      for (int64_t k = 0; k < v->n_elem[g]; ++k) {
        const int64_t e = v->elems[g][k];
        std::copy(mesh->elem_nodes + e * nn, mesh->elem_nodes + (e + 1) * nn, en.begin() + k * nn);
        std::copy(tag.begin() + e * nface, tag.begin() + (e + 1) * nface, fb.begin() + k * nface);
      }
      fr_mesh_desc cm = *mesh;
      cm.p = v->deg[g];
      cm.n_elem = v->n_elem[g];
      cm.elem_nodes = en.data();
      cm.face_bc = fb.data();
      cm.n_mesh = 1;
      cm.mesh_elem_begin = nullptr;
      fr_params cp = *prm;
      cp.n_probe = (int32_t)(gprobe[g].size() / d);
      cp.probe_xyz = cp.n_probe ? gprobe[g].data() : nullptr;
      cp.probe_mesh = nullptr;
      cp.max_samples = cp.n_probe ? prm->max_samples : 0;
      const fr_status st = build_solver(&cm, &cp, true, &v->child[g]);
      if (st != FR_OK) throw FrError(st, std::string("degree group ") + std::to_string(v->deg[g]) + ": " +
                                             fr_last_error());
      if (!get_dispatch(d, v->deg[g], prm->precision, v->dsp[g]))
        throw FrError(FR_ERR_UNSUPPORTED, "degree not compiled");
      const fr_solver *c = v->child[g];
      const int64_t nmort = c->nbnd - c->n_bc;
      int64_t want = 0;
      for (int64_t e : v->elems[g])
        for (int f = 0; f < nface; ++f)
          if (tag[(size_t)e * nface + f] == BC_MORTAR) want += c->Nfp;
      if (nmort != want) throw FrError(FR_ERR_MESH, "mortar point count mismatch");
      v->offset[g + 1] = (v->offset[g] + v->n_elem[g] * NV * c->Ns + STATE_ALIGN - 1) / STATE_ALIGN * STATE_ALIGN;
    }
    for (int g = v->n_group; g < MAX_GROUPS; ++g) v->offset[g + 1] = v->offset[g];
    VD_HIP_OK(hipGetDevice(&v->device));
    v->n_mortar = (int64_t)faces.size();
    v->faces = (MortarFace *)vd_upload(v, faces);
    if (v->precision == FR_FP64)
      upload_groups<double>(v, tab);
    else
      upload_groups<float>(v, tab);
    VD_HIP_OK(hipStreamCreateWithFlags(&v->cap_stream, hipStreamNonBlocking));
    const char *ng = std::getenv("FRMI_NO_GRAPH");
    v->use_graphs = (ng && ng[0] == '1') ? 0 : 1;
    VD_HIP_OK(hipDeviceSynchronize());
  } catch (const FrError &e) {
    vd_destroy(v);
    return vd_fail(e.code, e.what());
  } catch (const std::exception &e) {
    vd_destroy(v);
    return vd_fail(FR_ERR_OOM, e.what());
  }
  *out = v;
  return FR_OK;
}

fr_status fr_vdeg_groups(const fr_vdeg *v, int32_t *n_group, int32_t degree[5], int64_t n_elem[5], int64_t offset[6],
                         int64_t *n_mortar) {
  if (!v || !n_group || !degree || !n_elem || !offset || !n_mortar) return vd_fail(FR_ERR_ARG, "NULL argument");
  *n_group = v->n_group;
  for (int g = 0; g < MAX_GROUPS; ++g) {
    degree[g] = g < v->n_group ? v->deg[g] : -1;
    n_elem[g] = g < v->n_group ? v->n_elem[g] : 0;
  }
  for (int g = 0; g <= MAX_GROUPS; ++g) offset[g] = v->offset[g];
  *n_mortar = v->n_mortar;
  return FR_OK;
}

fr_status fr_vdeg_group_elems(const fr_vdeg *v, int32_t group, int64_t *elems) {
  if (!v || !elems) return vd_fail(FR_ERR_ARG, "NULL argument");
  if (group < 0 || group >= v->n_group) return vd_fail(FR_ERR_ARG, "group out of range");
  std::memcpy(elems, v->elems[group].data(), v->elems[group].size() * sizeof(int64_t));
  return FR_OK;
}

fr_status fr_vdeg_solpt_coords(const fr_vdeg *v, int32_t group, double *xyz) {
  if (!v || !xyz) return vd_fail(FR_ERR_ARG, "NULL argument");
  if (group < 0 || group >= v->n_group) return vd_fail(FR_ERR_ARG, "group out of range");
  const std::vector<double> &x = v->child[group]->xsol;
  std::memcpy(xyz, x.data(), x.size() * sizeof(double));
  return FR_OK;
}

fr_status fr_vdeg_rhs(fr_vdeg *v, const void *u, void *r, void *stream) {
  if (!v || !u || !r) return vd_fail(FR_ERR_ARG, "NULL argument");
  if (u == r) return vd_fail(FR_ERR_ARG, "u and r must not alias");
  try {
    vd_rhs(v, u, r, (hipStream_t)stream);
    VD_HIP_OK(hipGetLastError());
  } catch (const FrError &e) {
    return vd_fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return vd_fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_vdeg_rk_step(fr_vdeg *v, void *u, const double *dt, int32_t n_steps, int32_t sample_every,
                          void *stream) {
  if (!v || !u || !dt) return vd_fail(FR_ERR_ARG, "NULL argument");
  if (n_steps < 0 || sample_every < 0) return vd_fail(FR_ERR_ARG, "negative step count / sampling interval");
  hipStream_t st = (hipStream_t)stream;
  try {
    for (int32_t n = 0; n < n_steps; ++n) {
      const bool sample = sample_every > 0 && (v->steps_since_reset % sample_every) == 0;
      const bool fresh = n == 0;
      const int gi = (sample ? 1 : 0) + (fresh ? 2 : 0);
      if (v->use_graphs) {
        if (!v->graph[gi] || v->graph_u[gi] != u || v->graph_dt[gi] != dt) {
          if (v->graph[gi]) (void)hipGraphExecDestroy(v->graph[gi]);
          v->graph[gi] = nullptr;
          hipGraph_t g = nullptr;
          VD_HIP_OK(hipStreamBeginCapture(v->cap_stream, hipStreamCaptureModeRelaxed));
          vd_step(v, u, dt, sample, fresh, v->cap_stream);
          const hipError_t le = hipGetLastError();
          const hipError_t ce = hipStreamEndCapture(v->cap_stream, &g);
          if (le != hipSuccess)
            throw FrError(FR_ERR_HIP, std::string("launch during capture: ") + hipGetErrorString(le));
          VD_HIP_OK(ce);
          hipGraphExec_t ex = nullptr;
          const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          VD_HIP_OK(ie);
          v->graph[gi] = ex;
          v->graph_u[gi] = u;
          v->graph_dt[gi] = dt;
        }
        VD_HIP_OK(hipGraphLaunch(v->graph[gi], st));
      } else {
        vd_step(v, u, dt, sample, fresh, st);
        VD_HIP_OK(hipGetLastError());
      }
      v->steps_since_reset++;
    }
  } catch (const FrError &e) {
    return vd_fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return vd_fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_vdeg_reset_accumulators(fr_vdeg *v, void *stream) {
  if (!v) return vd_fail(FR_ERR_ARG, "NULL solver");
  for (int g = 0; g < v->n_group; ++g) {
    const fr_status st = fr_reset_accumulators(v->child[g], stream);
    if (st != FR_OK) return st;
  }
  v->steps_since_reset = 0;
  return FR_OK;
}

fr_status fr_vdeg_probe_series(fr_vdeg *v, double *series, int64_t cap, int64_t *n, void *stream) {
  if (!v || !n) return vd_fail(FR_ERR_ARG, "NULL argument");
  if (cap < 0 || (cap > 0 && !series)) return vd_fail(FR_ERR_ARG, "bad series buffer");
  *n = 0;
  for (int g = 0; g < v->n_group; ++g) {
    const fr_solver *c = v->child[g];
    // the group's series, strided by what it keeps (not by the caller's capacity)
    const int64_t cc = c->n_probe ? std::min<int64_t>(cap, c->cap) : 0;
    std::vector<double> buf((size_t)std::max(1, c->n_probe) * std::max<int64_t>(cc, 1));
    int64_t ng = 0;
    const fr_status st = fr_probe_series(v->child[g], cc ? buf.data() : nullptr, cc, &ng, stream);
    if (st != FR_OK) return st;
    *n = ng;
    const int64_t k = std::min<int64_t>(ng, cc);
    for (int a = 0; a < v->n_probe; ++a)
      if (v->probe_group[a] == g)
        for (int64_t j = 0; j < k; ++j) series[a * cap + j] = buf[(size_t)v->probe_slot[a] * cc + j];
  }
  return FR_OK;
}

fr_status fr_vdeg_mean_force(fr_vdeg *v, double *mean_force, int64_t *n_samples, void *stream) {
  if (!v || !mean_force) return vd_fail(FR_ERR_ARG, "NULL argument");
  if (!v->forces) return vd_fail(FR_ERR_ARG, "wall forces are not accumulated by this solver (forces = 0)");
  for (int j = 0; j < v->dim; ++j) mean_force[j] = 0.0;
  for (int g = 0; g < v->n_group; ++g) {
    double f[3] = {0.0, 0.0, 0.0};
    int64_t ns = 0;
    const fr_status st = fr_probe_oaspl(v->child[g], 1.0, nullptr, nullptr, f, &ns, stream);
    if (st != FR_OK) return st;
    for (int j = 0; j < v->dim; ++j) mean_force[j] += f[j];
    if (n_samples) *n_samples = ns;
  }
  return FR_OK;
}

void fr_vdeg_destroy(fr_vdeg *v) { vd_destroy(v); }

}  // extern "C"
