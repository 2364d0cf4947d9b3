// C ABI of libfrmi: argument validation, device allocation / upload, RK4 step sequencing with
// HIP graph replay, and the host-side OASPL arithmetic of Eqs. (9)-(12).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fr.h"
#include "fr_dispatch.hpp"

using namespace frmi;

namespace {
thread_local std::string g_err;

fr_status fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIP_OK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw FrError(e_ == hipErrorOutOfMemory ? FR_ERR_OOM : FR_ERR_HIP,                     \
                    std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

// Work area of fr_rhs_vjp_noalloc: one per GPU, held until the process ends.  In host code the
// array's name is only a host-side stand-in; its device address is taken once per device with
// hipGetSymbolAddress at solver set-up and only that address is handed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)FR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// device address of this device's scratch array (the device must be current); taken once per device
void acquire_scratch(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) throw FrError(FR_ERR_UNSUPPORTED, "device index beyond 64");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    throw FrError(FR_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch_ptr[dev] = p;
}

void *scratch_of(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (dev >= 0 && dev < MAX_DEVICES) ? g_scratch_ptr[dev] : nullptr;
}

// Autotuner choices of this process, keyed by what decides them: dimension, degree, precision,
// equations, LDG form, kernel kind and the mesh size's power of two
struct TuneKey {
  int dim, p, precision, equations, side, kind, bucket;
  bool operator<(const TuneKey &o) const {
    const int a[7] = {dim, p, precision, equations, side, kind, bucket};
    const int b[7] = {o.dim, o.p, o.precision, o.equations, o.side, o.kind, o.bucket};
    for (int i = 0; i < 7; ++i)
      if (a[i] != b[i]) return a[i] < b[i];
    return false;
  }
};
struct TuneEntry {
  int choice = 0;
  double ms[FR_TUNE_MAX] = {};
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune_cache;

TuneKey tune_key(const fr_solver *s, int kind) {
  int bucket = 0;
  while (((int64_t)1 << (bucket + 1)) <= s->Ne) ++bucket;
  const int side = s->precision == FR_FP64 ? ldg_side_of<double>(s->beta) : ldg_side_of<float>(s->beta);
  return TuneKey{s->dim, s->p, s->precision, s->equations, side, kind, bucket};
}

void *dalloc(fr_solver *s, size_t bytes) {
  void *p = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw FrError(FR_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  s->owned.push_back(p);
  return p;
}

template <typename T>
void *upload(fr_solver *s, const std::vector<T> &h) {
  void *d = dalloc(s, h.size() * sizeof(T));
  if (!h.empty()) HIP_OK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

// upload FP64 host data in the state precision
void *upload_real(fr_solver *s, const std::vector<double> &h) {
  if (s->precision == FR_FP64) return upload(s, h);
  std::vector<float> f(h.begin(), h.end());
  return upload(s, f);
}

template <typename T>
void *upload_flow(fr_solver *s) {
  std::vector<FlowDev<T>> f(s->n_mesh);
  for (int m = 0; m < s->n_mesh; ++m) {
    f[m].rho = (T)s->h_rho[m];
    for (int j = 0; j < 3; ++j) f[m].v[j] = j < s->dim ? (T)s->h_vel[m * s->dim + j] : T(0);
    f[m].p = (T)s->h_p[m];
    f[m].mu = (T)s->h_mu[m];
  }
  return upload(s, f);
}

void free_graphs(fr_solver *s) {
  for (int k = 0; k < 4; ++k) {
    if (s->graph[k]) (void)hipGraphExecDestroy(s->graph[k]);
    s->graph[k] = nullptr;
    s->graph_u[k] = nullptr;
    s->graph_dt[k] = nullptr;
  }
  for (auto &g : s->seg_graphs)
    if (g.ex) (void)hipGraphExecDestroy(g.ex);
  s->seg_graphs.clear();
}

void destroy(fr_solver *s) {
  if (!s) return;
  free_graphs(s);
  for (auto &r : s->prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : s->prof_pool) (void)hipEventDestroy(e);
  for (void *p : s->owned) (void)hipFree(p);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

// mesh-node adjoint tables and work arrays, on first use
void ensure_geo(fr_solver *s) {
  if (s->geo_Gm) return;
  MeshIn m;
  m.dim = s->dim;
  m.p = s->p;
  m.q = s->geom_q;
  m.n_elem = s->Ne;
  m.n_node = s->n_node;
  m.node_xyz = s->h_node_xyz.data();
  m.elem_nodes = s->h_elem_nodes.data();
  GeoAdj g = build_geo_adj(m, s->ops);
  if (g.nn != s->geo_nn) throw FrError(FR_ERR_MESH, "inconsistent geometry degree");
  const size_t T = s->tsize;
  s->geo_Xe = (double *)upload(s, g.Xe);
  s->geo_dphi_s = (double *)upload(s, g.dphi_s);
  s->geo_dphi_f = (double *)upload(s, g.dphi_f);
  s->geo_inc_ptr = (int32_t *)upload(s, g.inc_ptr);
  s->geo_inc = (int32_t *)upload(s, g.inc);
  s->geo_Xeb = (double *)dalloc(s, (size_t)s->Ne * g.nn * s->dim * sizeof(double));
  s->geo_R = dalloc(s, (size_t)s->Ne * s->NV * s->Ns * T);
  s->geo_Gn = dalloc(s, (size_t)s->Ne * (s->dim + 1) * s->Nf * T);
  s->geo_Gm = dalloc(s, (size_t)s->Ne * (s->dim * s->dim + 1) * s->Ns * T);
}

void zero_geo(fr_solver *s, hipStream_t st) {
  launch_fill_state(s, s->geo_Gm, s->Ne * (s->dim * s->dim + 1) * s->Ns, st);
  launch_fill_state(s, s->geo_Gn, s->Ne * (s->dim + 1) * s->Nf, st);
}

Dispatch dispatch_of(const fr_solver *s) {
  Dispatch d{};
  if (!get_dispatch(s->dim, s->p, s->precision, d)) throw FrError(FR_ERR_UNSUPPORTED, "unsupported (dim, p)");
  return d;
}
}  // namespace

extern "C" {

const char *fr_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace frmi {
fr_status set_error(int code, const std::string &msg) { return fail(code, msg); }

// One solver.  group: a degree group of a mesh with several solution degrees (degree 0 allowed,
// BC_MORTAR faces allowed; built by fr_vdeg_build, never returned through fr_build_operators).
fr_status build_solver(const fr_mesh_desc *mesh, const fr_params *prm, bool group, fr_solver **out) {
  if (!out) return fail(FR_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!mesh || !prm) return fail(FR_ERR_ARG, "mesh or params is NULL");
  if (mesh->dim != 2 && mesh->dim != 3) return fail(FR_ERR_ARG, "dim must be 2 or 3");
  if (mesh->p < (group ? 0 : 1) || mesh->p > 4)
    return fail(FR_ERR_UNSUPPORTED, group ? "degree must be in 0..4" : "p must be in 1..4");
  if (mesh->geom_q < 1 || mesh->geom_q > 4) return fail(FR_ERR_UNSUPPORTED, "geom_q must be in 1..4");
  if (mesh->n_elem <= 0 || mesh->n_node <= 0 || !mesh->node_xyz || !mesh->elem_nodes || !mesh->face_bc)
    return fail(FR_ERR_ARG, "empty mesh or NULL mesh array");
  if (mesh->n_periodic < 0 || (mesh->n_periodic > 0 && !mesh->periodic_vec))
    return fail(FR_ERR_ARG, "bad periodic vectors");
  const int n_mesh = mesh->n_mesh <= 0 ? 1 : mesh->n_mesh;
  if (mesh->n_mesh > 1 && !mesh->mesh_elem_begin) return fail(FR_ERR_ARG, "mesh_elem_begin is NULL");
  if (prm->equations != FR_EULER && prm->equations != FR_NAVIER_STOKES) return fail(FR_ERR_ARG, "bad equations");
  if (prm->precision != FR_FP64 && prm->precision != FR_FP32) return fail(FR_ERR_ARG, "bad precision");
  if (!prm->rho_inf || !prm->vel_inf || !prm->p_inf || !prm->mu) return fail(FR_ERR_ARG, "NULL free-stream array");
  if (!(prm->gamma > 1.0) || !(prm->prandtl > 0.0)) return fail(FR_ERR_ARG, "bad gamma / prandtl");
  if (prm->n_probe < 0 || (prm->n_probe > 0 && (!prm->probe_xyz || prm->max_samples <= 0)))
    return fail(FR_ERR_ARG, "bad probe arguments");
  fr_solver *s = new (std::nothrow) fr_solver();
  if (!s) return fail(FR_ERR_OOM, "host allocation failed");
  try {
    s->dim = mesh->dim;
    s->p = mesh->p;
    s->P = mesh->p + 1;
    s->NV = mesh->dim + 2;
    s->Ns = mesh->dim == 2 ? s->P * s->P : s->P * s->P * s->P;
    s->Nfp = mesh->dim == 2 ? s->P : s->P * s->P;
    s->Nf = 2 * mesh->dim * s->Nfp;
    s->Ne = mesh->n_elem;
    s->n_mesh = n_mesh;
    s->equations = prm->equations;
    s->precision = prm->precision;
    s->tsize = prm->precision == FR_FP64 ? 8 : 4;
    s->gamma = prm->gamma;
    s->prandtl = prm->prandtl;
    s->beta = prm->ldg_beta;
    s->tau = prm->ldg_tau;
    Dispatch dsp;
    if (!get_dispatch(s->dim, s->p, s->precision, dsp)) throw FrError(FR_ERR_UNSUPPORTED, "unsupported (dim, p)");
    MeshIn m;
    m.dim = mesh->dim;
    m.p = mesh->p;
    m.q = mesh->geom_q;
    m.n_elem = mesh->n_elem;
    m.n_node = mesh->n_node;
    m.node_xyz = mesh->node_xyz;
    m.elem_nodes = mesh->elem_nodes;
    m.face_bc = mesh->face_bc;
    m.n_periodic = mesh->n_periodic;
    m.periodic_vec = mesh->periodic_vec;
    m.n_mesh = n_mesh;
    m.allow_mortar = group;
    if (mesh->n_mesh > 1 || mesh->mesh_elem_begin) {
      m.mesh_begin.assign(mesh->mesh_elem_begin, mesh->mesh_elem_begin + n_mesh + 1);
      if (m.mesh_begin[0] != 0 || m.mesh_begin[n_mesh] != mesh->n_elem) throw FrError(FR_ERR_ARG, "bad mesh ranges");
      for (int k = 0; k < n_mesh; ++k)
        if (m.mesh_begin[k + 1] <= m.mesh_begin[k]) throw FrError(FR_ERR_ARG, "empty or unordered mesh range");
    } else {
      m.mesh_begin = {0, mesh->n_elem};
    }
    s->mesh_begin = m.mesh_begin;
    for (int k = 0; k < n_mesh; ++k) {
      if (!(prm->rho_inf[k] > 0.0) || !(prm->p_inf[k] > 0.0) || prm->mu[k] < 0.0)
        throw FrError(FR_ERR_ARG, "bad free stream");
      s->h_rho.push_back(prm->rho_inf[k]);
      s->h_p.push_back(prm->p_inf[k]);
      s->h_mu.push_back(prm->mu[k]);
      for (int j = 0; j < s->dim; ++j) s->h_vel.push_back(prm->vel_inf[k * s->dim + j]);
    }
    s->ops = build_ops_1d(s->p);
    Geometry g = build_geometry(m, s->ops);
    Connectivity c = build_connectivity(m, s->ops, g);
    // probes (located before any device allocation)
    s->n_probe = prm->n_probe;
    s->cap = prm->n_probe > 0 ? prm->max_samples : 1;
    s->forces = (prm->forces && s->equations == FR_NAVIER_STOKES) ? 1 : 0;
    std::vector<int64_t> pe, pnodes;
    std::vector<double> pw, pinf, pdw, pdxi;
    for (int a = 0; a < prm->n_probe; ++a) {
      int pm = prm->probe_mesh ? prm->probe_mesh[a] : 0;
      if (pm < 0 || pm >= n_mesh) throw FrError(FR_ERR_ARG, "probe mesh out of range");
      Probe pr = locate_probe(m, s->ops, prm->probe_xyz + (size_t)a * s->dim, pm);
      pe.push_back(pr.elem);
      pw.insert(pw.end(), pr.weights.begin(), pr.weights.end());
      pdw.insert(pdw.end(), pr.dweights.begin(), pr.dweights.end());
      pdxi.insert(pdxi.end(), pr.dxi.begin(), pr.dxi.end());
      pnodes.insert(pnodes.end(), pr.nodes.begin(), pr.nodes.end());
      pinf.push_back(prm->p_inf[pm]);
    }
    // host copy of the mesh for the mesh-node adjoint
    {
      int nn = 1;
      for (int k = 0; k < s->dim; ++k) nn *= mesh->geom_q + 1;
      s->geom_q = mesh->geom_q;
      s->n_node = mesh->n_node;
      s->geo_nn = nn;
      s->h_node_xyz.assign(mesh->node_xyz, mesh->node_xyz + mesh->n_node * s->dim);
      s->h_elem_nodes.assign(mesh->elem_nodes, mesh->elem_nodes + mesh->n_elem * nn);
    }
    s->xsol = std::move(g.xsol);
    // device work starts here (host-side validation of the mesh and probes is done)
    HIP_OK(hipGetDevice(&s->device));
    acquire_scratch(s->device);
    s->metric = upload_real(s, g.metric);
    g.metric.clear();
    g.metric.shrink_to_fit();
    s->npair = (int64_t)c.pairL.size();
    s->nbnd = (int64_t)c.bnd.size();
    s->n_wall = c.n_wall;
    s->n_bc = c.n_bc;
    s->pairL = (int32_t *)upload(s, c.pairL);
    s->pairR = (int32_t *)upload(s, c.pairR);
    s->bnd = (int32_t *)upload(s, c.bnd);
    s->pair_nrm = upload_real(s, c.pair_nrm);
    s->bnd_nrm = upload_real(s, c.bnd_nrm);
    s->bnd_w = (double *)upload(s, c.bnd_w);
    s->elem_mesh = (int32_t *)upload(s, c.elem_mesh);
    s->nbr = (int32_t *)upload(s, c.nbr);
    s->fnrm = upload_real(s, c.fnrm);
    s->h_wall_mesh_begin = c.wall_mesh_begin;
    s->wall_mesh_begin = (int64_t *)upload(s, c.wall_mesh_begin);
    s->flow = s->precision == FR_FP64 ? upload_flow<double>(s) : upload_flow<float>(s);
    const size_t T = s->tsize;
    const size_t nsol = (size_t)s->Ne * s->NV * s->Ns;
    // u_f by face; where face blocks are line-sized (uf_face_skip) the stage kernels write only
    // the faces something reads later: with the one-sided LDG the side whose values the flux side
    // takes, and boundary faces (wall force); otherwise (small blocks, two-sided LDG, Euler: the
    // face kernel reads both sides) every face
    {
      const int nface = 2 * s->dim;
      const size_t fs = (size_t)uf_face_stride(s->NV * s->Nfp, (int)T);
      s->uf = dalloc(s, (size_t)s->Ne * nface * fs * T);
      const int side = s->precision == FR_FP64 ? ldg_side_of<double>(s->beta) : ldg_side_of<float>(s->beta);
      const uint8_t all = (uint8_t)((1u << nface) - 1u);
      std::vector<uint8_t> faces((size_t)s->Ne, all);
      if (s->equations == FR_NAVIER_STOKES && side != 0 && uf_face_skip(s->NV * s->Nfp, (int)T)) {
        for (int64_t e = 0; e < s->Ne; ++e) {
          uint8_t m = 0;
          for (int f = 0; f < nface; ++f) {
            const int32_t code = c.nbr[(size_t)e * s->Nf + (size_t)f * s->Nfp];
            const bool isR = code >= 0 && (code & NBR_R_BIT) != 0;
            if (code < 0 || isR == (side < 0)) m |= (uint8_t)(1u << f);
          }
          faces[(size_t)e] = m;
        }
      }
      s->uf_faces = (uint8_t *)upload(s, faces);
    }
    s->fhat = dalloc(s, (size_t)s->Ne * 2 * s->dim * (size_t)uf_face_stride(s->NV * s->Nfp, (int)T) * T);
    s->acc = dalloc(s, nsol * T);
    s->ustage = dalloc(s, nsol * T);
    if (s->equations == FR_NAVIER_STOKES) {
      s->fvn = dalloc(s, (size_t)s->Ne * 2 * s->dim * (size_t)uf_face_stride(s->NV * s->Nfp, (int)T) * T);
      s->vol = dalloc(s, nsol * T);
    }
    if (s->nbnd > s->n_bc) s->ifc_uh = dalloc(s, (size_t)(s->nbnd - s->n_bc) * s->NV * T);
    s->h_probe_pinf = pinf;
    s->probe_elem = (int64_t *)upload(s, pe);
    s->probe_w = (double *)upload(s, pw);
    s->probe_pinf = (double *)upload(s, pinf);
    s->probe_dw = (double *)upload(s, pdw);
    s->probe_dxi = (double *)upload(s, pdxi);
    s->probe_nodes = (int64_t *)upload(s, pnodes);
    s->probe_coef = (double *)dalloc(s, (size_t)std::max(1, s->n_probe) * (s->NV + s->dim) * sizeof(double));
    s->series = (double *)dalloc(s, (size_t)std::max(1, s->n_probe) * s->cap * sizeof(double));
    s->sums = (double *)dalloc(s, (size_t)std::max(1, s->n_probe) * 2 * sizeof(double));
    s->force_acc = (double *)dalloc(s, (size_t)n_mesh * s->dim * sizeof(double));
    {
      int64_t mx = 0;
      for (int k = 0; k < n_mesh; ++k) mx = std::max(mx, c.wall_mesh_begin[k + 1] - c.wall_mesh_begin[k]);
      s->wall_nchunk = (int)std::max<int64_t>(1, (mx + WALL_CHUNK - 1) / WALL_CHUNK);
      s->wall_partial = (double *)dalloc(s, (size_t)n_mesh * s->wall_nchunk * s->dim * sizeof(double));
    }
    s->count = (unsigned long long *)dalloc(s, 2 * sizeof(unsigned long long));  // sample index, probe ticket
    s->nonfinite = (int *)dalloc(s, sizeof(int));
    HIP_OK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    const char *ng = std::getenv("FRMI_NO_GRAPH");
    s->use_graphs = (ng && ng[0] == '1') ? 0 : 1;
    fr_status st = fr_reset_accumulators(s, nullptr);
    if (st != FR_OK) throw FrError(st, g_err);
    HIP_OK(hipDeviceSynchronize());
  } catch (const FrError &e) {
    destroy(s);
    return fail(e.code, e.what());
  } catch (const std::exception &e) {
    destroy(s);
    return fail(FR_ERR_OOM, e.what());
  }
  *out = s;
  g_err.clear();
  return FR_OK;
}
}  // namespace frmi

extern "C" {

fr_status fr_build_operators(const fr_mesh_desc *mesh, const fr_params *prm, fr_solver **out) {
  return build_solver(mesh, prm, false, out);
}

fr_status fr_state_shape(const fr_solver *s, int64_t shape[3]) {
  if (!s || !shape) return fail(FR_ERR_ARG, "NULL argument");
  shape[0] = s->Ne;
  shape[1] = s->NV;
  shape[2] = s->Ns;
  return FR_OK;
}

fr_status fr_solpt_coords(const fr_solver *s, double *xyz) {
  if (!s || !xyz) return fail(FR_ERR_ARG, "NULL argument");
  std::memcpy(xyz, s->xsol.data(), s->xsol.size() * sizeof(double));
  return FR_OK;
}

fr_status fr_rhs(fr_solver *s, const void *u, void *r, void *stream) {
  if (!s || !u || !r) return fail(FR_ERR_ARG, "NULL argument");
  if (u == r) return fail(FR_ERR_ARG, "u and r must not alias");
  try {
    Dispatch d = dispatch_of(s);
    d.rhs(s, u, r, (hipStream_t)stream);
    HIP_OK(hipGetLastError());
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_rk_step(fr_solver *s, void *u, const double *dt, int32_t n_steps, int32_t sample_every, void *stream) {
  if (!s || !u || !dt) return fail(FR_ERR_ARG, "NULL argument");
  if (n_steps < 0 || sample_every < 0) return fail(FR_ERR_ARG, "negative step count / sampling interval");
  hipStream_t st = (hipStream_t)stream;
  try {
    Dispatch d = dispatch_of(s);
    for (int32_t n = 0; n < n_steps; ++n) {
      const bool sample = sample_every > 0 && (s->steps_since_reset % sample_every) == 0;
      const bool fresh = n == 0;  // later steps of this call reuse the u_f written by the last stage
      const int gi = (sample ? 1 : 0) + (fresh ? 2 : 0);
      if (s->use_graphs && !s->profiling) {
        if (!s->graph[gi] || s->graph_u[gi] != u || s->graph_dt[gi] != dt) {
          if (s->graph[gi]) (void)hipGraphExecDestroy(s->graph[gi]);
          s->graph[gi] = nullptr;
          hipGraph_t g = nullptr;
          HIP_OK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed));
          d.step(s, u, dt, sample, fresh, s->cap_stream);
          hipError_t le = hipGetLastError();
          hipError_t ce = hipStreamEndCapture(s->cap_stream, &g);
          if (le != hipSuccess) throw FrError(FR_ERR_HIP, std::string("launch during capture: ") + hipGetErrorString(le));
          HIP_OK(ce);
          hipGraphExec_t ex = nullptr;
          hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          HIP_OK(ie);
          s->graph[gi] = ex;
          s->graph_u[gi] = u;
          s->graph_dt[gi] = dt;
        }
        HIP_OK(hipGraphLaunch(s->graph[gi], st));
      } else {
        d.step(s, u, dt, sample, fresh, st);
        HIP_OK(hipGetLastError());
      }
      s->steps_since_reset++;
    }
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_reset_accumulators(fr_solver *s, void *stream) {
  if (!s) return fail(FR_ERR_ARG, "NULL solver");
  hipStream_t st = (hipStream_t)stream;
  try {
    launch_fill(s->series, (int64_t)std::max(1, s->n_probe) * s->cap, 0.0, st);
    launch_fill(s->sums, (int64_t)std::max(1, s->n_probe) * 2, 0.0, st);
    launch_fill(s->force_acc, (int64_t)s->n_mesh * s->dim, 0.0, st);
    launch_reset_counters(s->count, s->nonfinite, st);
    HIP_OK(hipGetLastError());
    s->steps_since_reset = 0;
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_force_coefficients(fr_solver *s, int32_t n_dir, const double *dirs, const double *ref_area,
                                double *coef, void *stream) {
  if (!s || !dirs || !ref_area || !coef || n_dir < 1) return fail(FR_ERR_ARG, "NULL argument or n_dir < 1");
  if (!s->forces) return fail(FR_ERR_ARG, "wall forces are not accumulated by this solver (forces = 0)");
  try {
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    unsigned long long cnt = 0;
    std::vector<double> frc((size_t)s->n_mesh * s->dim);
    HIP_OK(hipMemcpy(&cnt, s->count, sizeof(cnt), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(frc.data(), s->force_acc, frc.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (cnt == 0) return fail(FR_ERR_ARG, "no samples taken since the last reset");
    for (int m = 0; m < s->n_mesh; ++m) {
      double u2 = 0.0;
      for (int j = 0; j < s->dim; ++j) u2 += s->h_vel[(size_t)m * s->dim + j] * s->h_vel[(size_t)m * s->dim + j];
      const double q = 0.5 * s->h_rho[m] * u2;
      if (!(q > 0.0) || !(ref_area[m] > 0.0))
        return fail(FR_ERR_ARG, "mesh " + std::to_string(m) + ": free-stream dynamic pressure and reference area "
                                "must be positive");
      for (int k = 0; k < n_dir; ++k) {
        const double *e = dirs + ((size_t)m * n_dir + k) * s->dim;
        double f = 0.0;
        for (int j = 0; j < s->dim; ++j) f += frc[(size_t)m * s->dim + j] / (double)cnt * e[j];
        coef[(size_t)m * n_dir + k] = f / (q * ref_area[m]);
      }
    }
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_probe_series(fr_solver *s, double *series, int64_t cap, int64_t *n, void *stream) {
  if (!s || !n) return fail(FR_ERR_ARG, "NULL argument");
  if (cap < 0 || (cap > 0 && !series)) return fail(FR_ERR_ARG, "bad series buffer");
  try {
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    unsigned long long cnt = 0;
    HIP_OK(hipMemcpy(&cnt, s->count, sizeof(cnt), hipMemcpyDeviceToHost));
    *n = (int64_t)cnt;
    const int64_t k = std::min<int64_t>({(int64_t)cnt, (int64_t)s->cap, cap});
    std::vector<double> h((size_t)std::max(1, s->n_probe) * s->cap);
    if (s->n_probe > 0 && k > 0) {
      HIP_OK(hipMemcpy(h.data(), s->series, h.size() * sizeof(double), hipMemcpyDeviceToHost));
      for (int a = 0; a < s->n_probe; ++a)
        for (int64_t j = 0; j < k; ++j) series[a * cap + j] = h[(size_t)a * s->cap + j];
    }
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_probe_oaspl(fr_solver *s, double p_ref, double *prms, double *oaspl, double *mean_force,
                         int64_t *n_samples, void *stream) {
  if (!s) return fail(FR_ERR_ARG, "NULL solver");
  if (oaspl && !(p_ref > 0.0)) return fail(FR_ERR_ARG, "p_ref must be positive");
  try {
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    unsigned long long cnt = 0;
    int nf = 0;
    HIP_OK(hipMemcpy(&cnt, s->count, sizeof(cnt), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&nf, s->nonfinite, sizeof(int), hipMemcpyDeviceToHost));
    if (n_samples) *n_samples = (int64_t)cnt;
    const int np = std::max(1, s->n_probe);
    std::vector<double> sums((size_t)np * 2), ser((size_t)np * s->cap), frc((size_t)s->n_mesh * s->dim);
    HIP_OK(hipMemcpy(sums.data(), s->sums, sums.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(frc.data(), s->force_acc, frc.size() * sizeof(double), hipMemcpyDeviceToHost));
    const bool whole = cnt > 0 && cnt <= (unsigned long long)s->cap;
    if (whole && s->n_probe > 0)
      HIP_OK(hipMemcpy(ser.data(), s->series, ser.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int a = 0; a < s->n_probe; ++a) {
      double r = 0.0;
      if (cnt > 0) {
        if (whole) {  // two-pass over the stored FP64 series: population RMS about the mean
          double m1 = 0.0;
          for (unsigned long long k = 0; k < cnt; ++k) m1 += ser[(size_t)a * s->cap + k];
          m1 /= (double)cnt;
          double m2 = 0.0;
          for (unsigned long long k = 0; k < cnt; ++k) {
            const double dp = ser[(size_t)a * s->cap + k] - m1;
            m2 += dp * dp;
          }
          r = std::sqrt(m2 / (double)cnt);
        } else {  // from the FP64 sums of (p - p_inf)
          const double m1 = sums[2 * a] / (double)cnt, m2 = sums[2 * a + 1] / (double)cnt;
          r = std::sqrt(std::max(0.0, m2 - m1 * m1));
        }
      }
      if (prms) prms[a] = r;
      if (oaspl) oaspl[a] = r > 0.0 ? 20.0 * std::log10(r / p_ref) : -INFINITY;
    }
    if (mean_force)
      for (size_t k = 0; k < frc.size(); ++k) mean_force[k] = cnt > 0 ? frc[k] / (double)cnt : 0.0;
    if (nf) return fail(FR_ERR_NONFINITE, "a sampled probe pressure is not finite");
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_rhs_vjp_noalloc(fr_solver *s, const void *u, const void *r_bar, void *u_bar, void *stream) {
  if (!s || !u || !r_bar || !u_bar) return fail(FR_ERR_ARG, "NULL argument");
  if (u_bar == u || u_bar == r_bar) return fail(FR_ERR_ARG, "u_bar must not alias u or r_bar");
  const size_t need = vjp_work_elems(s) * s->tsize;
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(FR_ERR_ARG, "fr_rhs_vjp_noalloc needs " + std::to_string(need) + " bytes of work area; the static "
                            "buffer holds " + std::to_string(NOALLOC_SCRATCH_BYTES) + " (use fr_rhs_vjp)");
  void *work = scratch_of(s->device);
  if (!work) return fail(FR_ERR_HIP, "no scratch address for the solver's device");
  try {
    if (!launch_vjp(s, u, r_bar, u_bar, work, nullptr, nullptr, nullptr, 0.0, 0.0, nullptr, GeoVjpArgs{},
                    (hipStream_t)stream))
      throw FrError(FR_ERR_UNSUPPORTED, "unsupported (dim, p)");
    HIP_OK(hipGetLastError());
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_rhs_vjp(fr_solver *s, const void *u, const void *r_bar, void *u_bar, double *x_bar, void *stream) {
  if (!s || !u || !r_bar || !u_bar) return fail(FR_ERR_ARG, "NULL argument");
  if (u_bar == u || u_bar == r_bar) return fail(FR_ERR_ARG, "u_bar must not alias u or r_bar");
  hipStream_t st = (hipStream_t)stream;
  try {
    const size_t need = vjp_work_elems(s) * s->tsize;
    if (!s->vjp_work || s->vjp_bytes < need) {
      s->vjp_work = dalloc(s, need);  // kept until fr_destroy
      s->vjp_bytes = need;
    }
    GeoVjpArgs geo;
    if (x_bar) {
      if (s->geo_deferred) throw FrError(FR_ERR_ARG, "fr_rhs_vjp with x_bar inside a deferred node adjoint");
      ensure_geo(s);
      zero_geo(s, st);
      dispatch_of(s).rhs(s, u, s->geo_R, st);  // forward residual at u (adjoint of 1/J)
      geo = GeoVjpArgs{s->geo_Gm, s->geo_Gn, s->geo_R};
    }
    if (!launch_vjp(s, u, r_bar, u_bar, s->vjp_work, nullptr, nullptr, nullptr, 0.0, 0.0, nullptr, geo, st))
      throw FrError(FR_ERR_UNSUPPORTED, "unsupported (dim, p)");
    if (x_bar && !launch_geo_nodes(s, x_bar, st)) throw FrError(FR_ERR_UNSUPPORTED, "unsupported geometry degree");
    HIP_OK(hipGetLastError());
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_probe_vjp(fr_solver *s, const void *u, const double *p_bar, void *u_bar, double *x_bar, void *stream) {
  if (!s || !u || !u_bar || (s->n_probe > 0 && !p_bar)) return fail(FR_ERR_ARG, "NULL argument");
  try {
    Dispatch d = dispatch_of(s);
    d.probe_vjp(s, u, p_bar, u_bar, x_bar, (hipStream_t)stream);
    HIP_OK(hipGetLastError());
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_rk_step_stages(fr_solver *s, void *u, const double *dt, int32_t n_steps, void *states, void *stages,
                            void *residuals, void *stream) {
  if (!s || !u || !dt || !stages) return fail(FR_ERR_ARG, "NULL argument");
  if (n_steps < 1) return fail(FR_ERR_ARG, "n_steps must be >= 1");
  if (states == u || residuals == u) return fail(FR_ERR_ARG, "states / residuals must not alias u");
  try {
    Dispatch d = dispatch_of(s);
    d.step_record(s, u, dt, n_steps, states, stages, residuals, (hipStream_t)stream);
    HIP_OK(hipGetLastError());
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_rk_step_vjp(fr_solver *s, const void *u_n, const double *dt, const void *stages, const void *residuals,
                         void *u_bar, double *x_bar, void *stream) {
  if (!s || !u_n || !dt || !u_bar) return fail(FR_ERR_ARG, "NULL argument");
  if (u_bar == u_n) return fail(FR_ERR_ARG, "u_bar must not alias u_n");
  hipStream_t st = (hipStream_t)stream;
  try {
    Dispatch d = dispatch_of(s);
    const size_t nb = (size_t)s->Ne * s->NV * s->Ns * s->tsize;
    if (!s->adj_work) s->adj_work = (char *)dalloc(s, nb * 11);  // A, KB, Z, temp state, 3 stages, 4 residuals
    if (!s->vjp_work) {
      s->vjp_bytes = vjp_work_elems(s) * s->tsize;
      s->vjp_work = dalloc(s, s->vjp_bytes);
    }
    char *A = s->adj_work, *KB = A + nb, *Z = KB + nb, *TMP = Z + nb, *STG = TMP + nb, *RES = STG + 3 * nb;
    const char *Y = (const char *)stages;
    const char *Rs = (const char *)residuals;
    if (!Y) {  // recompute the stage states (and, for x_bar, the stage residuals) from u_n on a copy
      HIP_OK(hipMemcpyAsync(TMP, u_n, nb, hipMemcpyDeviceToDevice, st));
      d.step_record(s, TMP, dt, 1, nullptr, STG, x_bar ? RES : nullptr, st);
      Y = STG;
      if (x_bar) Rs = RES;
    }
    // u_{n+1} = u_n + dt/6 (k1 + 2 k2 + 2 k3 + k4); k_{s} = R(y_s), y1 = u_n, y2 = u_n + dt/2 k1,
    // y3 = u_n + dt/2 k2, y4 = u_n + dt k3.  Reverse, with a = u_bar on entry:
    //   k4_bar = dt/6 a;  z_s = (dR/du (y_s))^T k_s_bar;  u_bar += z_s;
    //   k_{s-1}_bar = dt (w_{s-1} a + c_{s-1} z_s)  with w = (1/6, 1/3, 1/3), c = (1/2, 1/2, 1)
    const void *ys[4] = {u_n, Y, Y + nb, Y + 2 * nb};
    const double cA[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const double cZ[4] = {0.5, 0.5, 1.0, 0.0};
    if (x_bar) {
      ensure_geo(s);
      if (!s->geo_deferred) zero_geo(s, st);
    }
    if (!x_bar || Rs) {  // the fused step sequence (stage residuals at hand when x_bar is wanted)
      const void *rs[4] = {nullptr, nullptr, nullptr, nullptr};
      if (x_bar)
        for (int k = 0; k < 4; ++k) rs[k] = Rs + (size_t)k * nb;
      if (!launch_vjp_rk_step(s, ys, u_bar, A, dt, x_bar ? rs : nullptr, x_bar ? s->geo_Gm : nullptr,
                              x_bar ? s->geo_Gn : nullptr, s->vjp_work, st))
        throw FrError(FR_ERR_UNSUPPORTED, "unsupported (dim, p)");
      if (x_bar && !s->geo_deferred && !launch_geo_nodes(s, x_bar, st))
        throw FrError(FR_ERR_UNSUPPORTED, "unsupported geometry degree");
      HIP_OK(hipGetLastError());
      return FR_OK;
    }
    d.rk_adj_combine(s, A, nullptr, KB, u_bar, Z, cA[3], 0.0, dt, st);  // A = a, KB = dt/6 a, Z = 0
    // each stage's VJP ends in the RK epilogue: u_bar += z_s, KB = k_{s-1}_bar; with x_bar the
    // metric adjoints of the four stages accumulate, then go to the nodes once
    for (int k = 3; k >= 0; --k) {
      GeoVjpArgs geo;
      if (x_bar) {
        const void *Rk = Rs ? (const void *)(Rs + (size_t)k * nb) : s->geo_R;
        if (!Rs) d.rhs(s, ys[k], s->geo_R, st);  // residual of stage k (adjoint of 1/J)
        geo = GeoVjpArgs{s->geo_Gm, s->geo_Gn, Rk};
      }
      if (!launch_vjp(s, ys[k], KB, Z, s->vjp_work, A, KB, u_bar, k > 0 ? cA[k - 1] : 0.0, k > 0 ? cZ[k - 1] : 0.0,
                      dt, geo, st))
        throw FrError(FR_ERR_UNSUPPORTED, "unsupported (dim, p)");
    }
    if (x_bar && !s->geo_deferred && !launch_geo_nodes(s, x_bar, st))
      throw FrError(FR_ERR_UNSUPPORTED, "unsupported geometry degree");
    HIP_OK(hipGetLastError());
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_rk_segment_vjp(fr_solver *s, const void *states, const double *dt, const void *stages,
                            const void *residuals, const double *p_bar, int32_t n_steps, void *u_bar, double *x_bar,
                            void *stream) {
  if (!s || !states || !dt || !stages || !u_bar || (s->n_probe > 0 && !p_bar))
    return fail(FR_ERR_ARG, "NULL argument");
  if (n_steps < 1) return fail(FR_ERR_ARG, "n_steps must be >= 1");
  if (x_bar && (!residuals || !s->geo_deferred))
    return fail(FR_ERR_ARG, "x_bar needs the stage residuals and fr_geo_adjoint_begin");
  hipStream_t st = (hipStream_t)stream;
  try {
    Dispatch d = dispatch_of(s);
    const size_t nb = (size_t)s->Ne * s->NV * s->Ns * s->tsize;
    // work areas exist before any capture
    if (!s->adj_work) s->adj_work = (char *)dalloc(s, nb * 11);
    if (!s->vjp_work) {
      s->vjp_bytes = vjp_work_elems(s) * s->tsize;
      s->vjp_work = dalloc(s, s->vjp_bytes);
    }
    if (x_bar) ensure_geo(s);
    auto body = [&](hipStream_t q) {
      const char *X = (const char *)states, *Y = (const char *)stages, *R = (const char *)residuals;
      for (int j = n_steps - 1; j >= 0; --j) {
        const char *yj = Y + (size_t)j * 3 * nb;
        const void *ys[4] = {X + (size_t)j * nb, yj, yj + nb, yj + 2 * nb};
        const void *rs[4] = {nullptr, nullptr, nullptr, nullptr};
        if (x_bar)
          for (int k = 0; k < 4; ++k) rs[k] = R + ((size_t)j * 4 + k) * nb;
        if (!launch_vjp_rk_step(s, ys, u_bar, s->adj_work, dt, x_bar ? rs : nullptr, x_bar ? s->geo_Gm : nullptr,
                                x_bar ? s->geo_Gn : nullptr, s->vjp_work, q))
          throw FrError(FR_ERR_UNSUPPORTED, "unsupported (dim, p)");
        d.probe_vjp(s, ys[0], p_bar ? p_bar + (size_t)j * s->n_probe : nullptr, u_bar, x_bar, q);
      }
    };
    if (!s->use_graphs || s->profiling) {
      body(st);
      HIP_OK(hipGetLastError());
      return FR_OK;
    }
    fr_solver::SegGraph *g = nullptr;
    for (auto &c : s->seg_graphs)
      if (c.states == states && c.stages == stages && c.res == residuals && c.pbar == p_bar && c.ubar == u_bar &&
          c.dt == dt && c.xbar == x_bar && c.n == n_steps)
        g = &c;
    if (!g) {
      if (s->seg_graphs.size() >= 8) {  // keep a handful (two record slots x full and tail segments)
        (void)hipGraphExecDestroy(s->seg_graphs.front().ex);
        s->seg_graphs.erase(s->seg_graphs.begin());
      }
      hipGraph_t gr = nullptr;
      HIP_OK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed));
      try {
        body(s->cap_stream);
      } catch (...) {
        (void)hipStreamEndCapture(s->cap_stream, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        throw;
      }
      const hipError_t le = hipGetLastError();
      const hipError_t ce = hipStreamEndCapture(s->cap_stream, &gr);
      if (le != hipSuccess) throw FrError(FR_ERR_HIP, std::string("launch during capture: ") + hipGetErrorString(le));
      HIP_OK(ce);
      hipGraphExec_t ex = nullptr;
      const hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      HIP_OK(ie);
      fr_solver::SegGraph c;
      c.ex = ex;
      c.states = states;
      c.stages = stages;
      c.res = residuals;
      c.pbar = p_bar;
      c.ubar = u_bar;
      c.dt = dt;
      c.xbar = x_bar;
      c.n = n_steps;
      s->seg_graphs.push_back(c);
      g = &s->seg_graphs.back();
    }
    HIP_OK(hipGraphLaunch(g->ex, st));
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_geo_adjoint_begin(fr_solver *s, void *stream) {
  if (!s) return fail(FR_ERR_ARG, "NULL solver");
  try {
    ensure_geo(s);
    zero_geo(s, (hipStream_t)stream);
    s->geo_deferred = 1;
    HIP_OK(hipGetLastError());
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_geo_adjoint_end(fr_solver *s, double *x_bar, void *stream) {
  if (!s || !x_bar) return fail(FR_ERR_ARG, "NULL argument");
  if (!s->geo_deferred) return fail(FR_ERR_ARG, "fr_geo_adjoint_begin was not called");
  hipStream_t st = (hipStream_t)stream;
  try {
    s->geo_deferred = 0;
    if (!launch_geo_nodes(s, x_bar, st)) throw FrError(FR_ERR_UNSUPPORTED, "unsupported geometry degree");
    HIP_OK(hipGetLastError());
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_autotune(fr_solver *s, const void *u, const double *dt, int32_t reps, int32_t kinds_mask,
                      int32_t *choice, double *ms, void *stream) {
  if (!s || !u || !dt) return fail(FR_ERR_ARG, "NULL argument");
  if (reps < 1) return fail(FR_ERR_ARG, "reps must be >= 1");
  if (kinds_mask < 0 || kinds_mask > 15) return fail(FR_ERR_ARG, "kinds_mask must be in 0..15");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a = nullptr, b = nullptr;
  void *tmp = nullptr, *work = nullptr, *tmp2 = nullptr;
  // restored if timing fails part way, so the solver keeps the candidates it had
  const int prof = s->profiling;
  int tune0[4];
  for (int k = 0; k < 4; ++k) tune0[k] = s->tune[k];
  try {
    Dispatch d = dispatch_of(s);
    const size_t nb = (size_t)s->Ne * s->NV * s->Ns * s->tsize;
    const int kinds_ns[3] = {0, 1, 3}, kinds_eu[1] = {2};
    const int *kinds = s->equations == FR_NAVIER_STOKES ? kinds_ns : kinds_eu;
    int32_t vc[FR_TUNE_MAX * 3];
    const int nk = s->equations == FR_NAVIER_STOKES ? (vjp_tune_cands(s, vc) > 0 ? 3 : 2) : 1;
    double times[4][FR_TUNE_MAX] = {};
    int cached[4] = {0, 0, 0, 0};
    auto cands_of = [&](int kind, int32_t *cand) { return kind == 3 ? vjp_tune_cands(s, cand) : d.tune_cands(kind, cand); };
    s->profiling = 0;
    for (int q = 0; q < nk; ++q) {
      const int kind = kinds[q];
      if (kinds_mask != 0 && !(kinds_mask & (1 << kind))) continue;
      int32_t cand[FR_TUNE_MAX * 3];
      const int nc = cands_of(kind, cand);
      const TuneKey key = tune_key(s, kind);
      {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
          s->tune[kind] = it->second.choice;
          for (int c = 0; c < FR_TUNE_MAX; ++c) times[kind][c] = it->second.ms[c];
          cached[kind] = 1;
          continue;
        }
      }
      if (!tmp) {
        HIP_OK(hipMalloc(&tmp, nb));
        HIP_OK(hipEventCreate(&a));
        HIP_OK(hipEventCreate(&b));
      }
      double best = 1e300;
      int best_c = 0;
      for (int c = 0; c < nc; ++c) {
        bool dup = false;  // tile halves and quarters coincide for small defaults
        for (int c2 = 0; c2 < c; ++c2)
          dup = dup || (cand[3 * c] == cand[3 * c2] && cand[3 * c + 1] == cand[3 * c2 + 1] &&
                        cand[3 * c + 2] == cand[3 * c2 + 2]);
        if (dup) continue;
        s->tune[kind] = c;
        HIP_OK(hipMemcpyAsync(tmp, u, nb, hipMemcpyDeviceToDevice, st));
        if (kind == 3) {  // the residual adjoint at u with r_bar = u (values do not matter for timing)
          if (!work) {
            HIP_OK(hipMalloc(&work, vjp_work_elems(s) * s->tsize));
            HIP_OK(hipMalloc(&tmp2, nb));
            HIP_OK(hipMemsetAsync(tmp2, 0, nb, st));  // u_bar accumulates: start from finite values
          }
          const GeoVjpArgs geo{};
          auto vjp = [&]() {
            if (!launch_vjp(s, u, tmp, tmp2, work, nullptr, nullptr, nullptr, 0.0, 0.0, nullptr, geo, st))
              throw FrError(FR_ERR_UNSUPPORTED, "adjoint not compiled for this degree");
          };
          vjp();  // warm-up
          HIP_OK(hipEventRecord(a, st));
          for (int r = 0; r < reps * 4; ++r) vjp();  // as many residual adjoints as forward stages
          HIP_OK(hipEventRecord(b, st));
        } else {
          d.step(s, tmp, dt, false, true, st);  // warm-up (first launch of this variant)
          HIP_OK(hipEventRecord(a, st));
          for (int r = 0; r < reps; ++r) d.step(s, tmp, dt, false, r == 0, st);
          HIP_OK(hipEventRecord(b, st));
        }
        HIP_OK(hipEventSynchronize(b));
        float t = 0.0f;
        HIP_OK(hipEventElapsedTime(&t, a, b));
        times[kind][c] = (double)t / reps;
        if (times[kind][c] < best) {
          best = times[kind][c];
          best_c = c;
        }
      }
      s->tune[kind] = best_c;
      std::lock_guard<std::mutex> lock(g_tune_mu);
      TuneEntry &en = g_tune_cache[key];
      en.choice = best_c;
      for (int c = 0; c < FR_TUNE_MAX; ++c) en.ms[c] = times[kind][c];
    }
    s->profiling = prof;
    free_graphs(s);  // captured steps must use the chosen candidates
    if (choice)
      for (int k = 0; k < 4; ++k) {
        int32_t cand[FR_TUNE_MAX * 3];
        const int nc = cands_of(k, cand);
        const int c = s->tune[k] < nc ? s->tune[k] : 0;
        choice[4 * k] = nc > 0 ? cand[3 * c] : 0;
        choice[4 * k + 1] = nc > 0 ? cand[3 * c + 1] : 0;
        choice[4 * k + 2] = nc > 0 ? cand[3 * c + 2] : 0;
        choice[4 * k + 3] = cached[k];
      }
    if (ms)
      for (int k = 0; k < 4; ++k)
        for (int c = 0; c < FR_TUNE_MAX; ++c) ms[k * FR_TUNE_MAX + c] = times[k][c];
    // every candidate run has ended (the last event was waited for); release the work areas
    const hipError_t rel[5] = {a ? hipEventDestroy(a) : hipSuccess, b ? hipEventDestroy(b) : hipSuccess,
                               tmp ? hipFree(tmp) : hipSuccess, work ? hipFree(work) : hipSuccess,
                               tmp2 ? hipFree(tmp2) : hipSuccess};
    a = b = nullptr;
    tmp = work = tmp2 = nullptr;
    for (const hipError_t r : rel) HIP_OK(r);
  } catch (const std::exception &ex) {
    (void)hipStreamSynchronize(st);  // no candidate run may still use the work areas
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (tmp) (void)hipFree(tmp);
    if (work) (void)hipFree(work);
    if (tmp2) (void)hipFree(tmp2);
    s->profiling = prof;
    for (int k = 0; k < 4; ++k) s->tune[k] = tune0[k];
    free_graphs(s);
    const FrError *fe = dynamic_cast<const FrError *>(&ex);
    return fail(fe ? fe->code : FR_ERR_OOM, ex.what());
  }
  return FR_OK;
}

fr_status fr_tune_candidates(const fr_solver *s, int32_t kind, int32_t *cand, int32_t *n) {
  if (!s || !cand || !n) return fail(FR_ERR_ARG, "NULL argument");
  if (kind < 0 || kind > 3) return fail(FR_ERR_ARG, "kind must be in 0..3");
  try {
    Dispatch d = dispatch_of(s);
    *n = kind == 3 ? vjp_tune_cands(s, cand) : d.tune_cands(kind, cand);
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

fr_status fr_tune_select(fr_solver *s, int32_t kind, int32_t index) {
  if (!s) return fail(FR_ERR_ARG, "NULL solver");
  if (kind < 0 || kind > 3) return fail(FR_ERR_ARG, "kind must be in 0..3");
  try {
    Dispatch d = dispatch_of(s);
    int32_t cand[FR_TUNE_MAX * 3];
    const int nc = kind == 3 ? vjp_tune_cands(s, cand) : d.tune_cands(kind, cand);
    if (index < 0 || index >= nc) return fail(FR_ERR_ARG, "candidate index out of range");
    s->tune[kind] = index;
    free_graphs(s);
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

void fr_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache.clear();
}

fr_status fr_solver_info(const fr_solver *s, int64_t info[8]) {
  if (!s || !info) return fail(FR_ERR_ARG, "NULL argument");
  info[0] = s->Ne;
  info[1] = s->NV;
  info[2] = s->Ns;
  info[3] = s->Nf;
  info[4] = s->npair;
  info[5] = s->nbnd;
  info[6] = s->n_wall;
  info[7] = s->n_mesh;
  return FR_OK;
}

fr_status fr_profile_enable(fr_solver *s, int32_t enable) {
  if (!s) return fail(FR_ERR_ARG, "NULL solver");
  s->profiling = enable ? 1 : 0;
  return FR_OK;
}

fr_status fr_profile_read(fr_solver *s, double *total_ms, int64_t *launches, void *stream) {
  if (!s || !total_ms || !launches) return fail(FR_ERR_ARG, "NULL argument");
  try {
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    for (auto &r : s->prof_pending) {
      float ms = 0.0f;
      HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
      if (r.id >= 0 && r.id < FR_K_COUNT) {
        s->prof_ms[r.id] += ms;
        s->prof_n[r.id] += 1;
      }
      s->prof_pool.push_back(r.a);
      s->prof_pool.push_back(r.b);
    }
    s->prof_pending.clear();
    for (int k = 0; k < FR_K_COUNT; ++k) {
      total_ms[k] = s->prof_ms[k];
      launches[k] = s->prof_n[k];
      s->prof_ms[k] = 0.0;
      s->prof_n[k] = 0;
    }
  } catch (const FrError &e) {
    return fail(e.code, e.what());
  } catch (const std::exception &e) {  // host allocation
    return fail(FR_ERR_OOM, e.what());
  }
  return FR_OK;
}

void fr_destroy(fr_solver *s) { destroy(s); }

}  // extern "C"
