// Host-side entry points of the kernel engines, shared by the API layer and the engines.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/fr.h"

#include "fr_solver.hpp"

namespace frmi {

// per (dim, p, precision) function table of the forward engine
struct Dispatch {
  void (*rhs)(const fr_solver *, const void *, void *, hipStream_t);
  void (*step)(const fr_solver *, void *, const double *, bool, bool, hipStream_t);
  // pieces of a residual / RK4 stage for degree-group solvers (part: 1 volume and common-flux
  // kernels, 2 lifting and RK kernel, 3 both)
  void (*interp)(const fr_solver *, const void *, hipStream_t);
  void (*sample_probes)(const fr_solver *, const void *, hipStream_t);
  void (*rhs_part)(const fr_solver *, const void *, void *, int, hipStream_t);
  void (*stage_k)(const fr_solver *, void *, const double *, int, bool, int, hipStream_t);
  void (*step_record)(const fr_solver *, void *, const double *, int, void *, void *, void *, hipStream_t);
  void (*probe_vjp)(const fr_solver *, const void *, const double *, void *, double *, hipStream_t);
  void (*rk_adj_combine)(const fr_solver *, void *, void *, void *, void *, void *, double, double,
                         const double *, hipStream_t);
  void (*zero)(const fr_solver *, void *, hipStream_t);
  // autotuner candidates of volume kernel `kind` (0: NS volume, 1: NS lifting + RK, 2: Euler
  // volume + RK): cand[c][3] = (elements per workgroup, waves-per-SIMD bound or 0 for the
  // default, engine: 0 vector ALU, 1 matrix cores); returns the count (<= FR_TUNE_MAX)
  int (*tune_cands)(int kind, int32_t *cand);
};
bool get_dispatch(int dim, int p, int precision, Dispatch &out);
// API layer (fr_api.hip): builds one solver (group: a degree group of a variable-degree mesh) and
// records an error message for fr_last_error
fr_status build_solver(const fr_mesh_desc *mesh, const fr_params *prm, bool group, fr_solver **out);
fr_status set_error(int code, const std::string &msg);
void launch_fill(double *p, int64_t n, double v, hipStream_t st);
void launch_fill_state(const fr_solver *s, void *p, int64_t n, hipStream_t st);
void launch_reset_counters(unsigned long long *count, int *nonfinite, hipStream_t st);

// adjoint engine (fr_vjp.hip)
size_t vjp_work_elems(const fr_solver *s);
// geometric adjoint arrays of one residual VJP: metric and normal adjoints accumulate (+=) into
// Gm / Gn; R is the forward residual at the linearisation state
struct GeoVjpArgs {
  void *Gm = nullptr, *Gn = nullptr;
  const void *R = nullptr;
};
bool launch_vjp(const fr_solver *s, const void *u, const void *rbar, void *ubar, void *work, const void *rk_a,
                void *rk_kb, void *rk_ub, double ca, double cz, const double *dt, const GeoVjpArgs &geo,
                hipStream_t st);

bool launch_vjp_rk_step(const fr_solver *s, const void *const ys[4], void *u_bar, void *A, const double *dt,
                        const void *const Rs[4], void *Gm, void *Gn, void *work, hipStream_t st);

// autotuner candidates of the NS volume adjoint (kind 3), as Dispatch::tune_cands; 0 if the
// adjoint is not compiled for the solver's degree
int vjp_tune_cands(const fr_solver *s, int32_t *cand);

// mesh-node adjoint (fr_geo.hip): x_bar += (d metrics / d X)^T (Gm, Gn)
bool launch_geo_nodes(const fr_solver *s, double *x_bar, hipStream_t st);

}  // namespace frmi
