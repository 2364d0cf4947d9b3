/*
 * fr.h -- C ABI of the MI355X flux-reconstruction residual / RK4 library (libfrmi.so).
 *
 * The library evaluates the explicit FR residual of the compressible Navier-Stokes
 * (or Euler) equations -- conservation law Eq. (1), conserved variables Eq. (2),
 * fluxes Eqs. (3)-(7) of the governing-equations subsection -- with the flux
 * reconstruction scheme named in the flow-solver subsection (Gauss-Legendre
 * solution/flux points, g_DG correction, Rusanov + LDG common fluxes, adiabatic
 * no-slip walls and Riemann-invariant far field as in the computational-details
 * paragraphs), advances it with classical RK4, and accumulates the probe-pressure
 * and wall-force statistics that feed Eqs. (8)-(12).
 *
 * Conventions shared by every entry point
 *  - Return value: FR_OK (0) or a negative fr_status.  No C++ exception crosses the
 *    ABI.  fr_last_error() gives a thread-local message for the last failure.
 *  - Arguments are validated before any launch; an invalid argument launches nothing.
 *  - "device" pointers are HIP device memory (e.g. torch CUDA tensors on ROCm);
 *    "host" pointers are ordinary CPU memory.  The caller owns every buffer it passes;
 *    the solver handle owns operators, metrics, connectivity, work arrays, HIP graphs
 *    and the FP64 accumulators.
 *  - State layout: element-major  u[n_elem][nv][Ns], contiguous, nv = dim + 2
 *    (rho, rho u_1..rho u_dim, rho E), Ns = (p+1)^dim solution points in lexicographic
 *    order (first reference coordinate fastest).  Element type: double for FR_FP64,
 *    float for FR_FP32 (the accumulators are always double).
 *  - `stream` is a hipStream_t (NULL = default stream).  All work is ordered on it;
 *    only fr_probe_oaspl / fr_probe_series / fr_solpt_coords synchronise it.
 *    Device faults surface as FR_ERR_HIP at the next synchronising call.
 *  - A handle is not thread safe; calls on one handle must not overlap.
 */
#ifndef FRMI_FR_H
#define FRMI_FR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fr_status;
#define FR_OK                0
#define FR_ERR_ARG          -1  /* null pointer, bad size / enum / range               */
#define FR_ERR_MESH         -2  /* non-positive Jacobian, unmatched face, probe outside */
#define FR_ERR_UNSUPPORTED  -3  /* (dim, p) combination not compiled                    */
#define FR_ERR_HIP          -4  /* HIP runtime error (launch, copy, device fault)       */
#define FR_ERR_NONFINITE    -5  /* a sampled probe pressure was NaN / Inf               */
#define FR_ERR_OOM          -6  /* device or host allocation failed                     */

/* face tags (per element face) */
#define FR_FACE_AUTO     0   /* matched geometrically with another face (conforming or periodic) */
#define FR_BC_WALL       1   /* adiabatic no-slip wall                                            */
#define FR_BC_FARFIELD   2   /* Riemann-invariant (characteristic) far field                      */

#define FR_EULER          0
#define FR_NAVIER_STOKES  1
#define FR_FP64           0
#define FR_FP32           1

typedef struct fr_solver fr_solver;  /* opaque, library-owned */

/*
 * Mesh description (host pointers, read during fr_build_operators only).
 *  dim 2|3; p 1..4 (solution degree); geom_q 1..4 geometry degree.
 *  node_xyz[n_node][dim]: physical node coordinates.
 *  elem_nodes[n_elem][(geom_q+1)^dim]: node ids at the tensor Gauss-Lobatto-Legendre
 *      points of degree geom_q of [-1,1]^dim, first reference coordinate fastest;
 *      elements must be right-handed (positive Jacobian) -> else FR_ERR_MESH.
 *  face_bc[n_elem][2*dim]: face f lies on reference coordinate f/2 at -1 (f even) or
 *      +1 (f odd); tag FR_FACE_AUTO / FR_BC_WALL / FR_BC_FARFIELD.
 *  periodic_vec[n_periodic][dim]: translations identifying FR_FACE_AUTO faces (nullable
 *      when n_periodic = 0).
 *  mesh_elem_begin[n_mesh+1]: disjoint element ranges of independent meshes advanced
 *      together (batched designs); NULL means one mesh [0, n_elem).
 */
typedef struct {
  int32_t dim, p, geom_q, n_periodic;
  int64_t n_elem, n_node;
  const double  *node_xyz;
  const int64_t *elem_nodes;
  const int32_t *face_bc;
  const double  *periodic_vec;
  int32_t        n_mesh;
  int32_t        reserved0;
  const int64_t *mesh_elem_begin;
} fr_mesh_desc;

/*
 * Physical and run parameters (host pointers, copied during fr_build_operators).
 *  equations FR_EULER | FR_NAVIER_STOKES; precision FR_FP64 | FR_FP32 (state, operators
 *  and fluxes; probe / force accumulators are FP64 in both).
 *  gamma (1.4), prandtl (0.71), ldg_beta (0.5), ldg_tau (penalty, 0.1).
 *  Per mesh m: rho_inf[m], vel_inf[m*dim + j], p_inf[m], mu[m] (constant viscosity).
 *  Probes: probe_xyz[n_probe][dim] located (lowest-index element containing it) in mesh
 *  probe_mesh[n_probe] (NULL -> mesh 0); FR_ERR_MESH if outside.  max_samples = capacity
 *  of the per-probe FP64 pressure series kept on the device.
 *  forces != 0 accumulates the wall force per mesh at each sample (NS only).
 */
typedef struct {
  int32_t equations, precision;
  double  gamma, prandtl, ldg_beta, ldg_tau;
  const double *rho_inf, *vel_inf, *p_inf, *mu;
  int32_t n_probe, max_samples;
  const double  *probe_xyz;
  const int32_t *probe_mesh;
  int32_t forces;
  int32_t reserved0;
} fr_params;

/* Build operators (Gauss-Legendre points, Lagrange derivative, interpolation and
 * g_DG correction-derivative tables), curved-element metrics at solution and flux
 * points, face connectivity (conforming, periodic, wall, far field), probe tables, and
 * allocate the device work arrays.  *out receives the handle (NULL on failure). */
fr_status fr_build_operators(const fr_mesh_desc *mesh, const fr_params *params, fr_solver **out);

/* shape[0..2] = {n_elem, nv, Ns} of a state array. */
fr_status fr_state_shape(const fr_solver *s, int64_t shape[3]);

/* Physical coordinates of the solution points, host out xyz[n_elem][Ns][dim] (FP64). */
fr_status fr_solpt_coords(const fr_solver *s, double *xyz);

/* r = R(u) = -(1/J)[div F~ + correction], the FR residual (du/dt).  u, r: device state
 * arrays (may not alias). */
fr_status fr_rhs(fr_solver *s, const void *u, void *r, void *stream);

/* Advance u (device state, in place) by n_steps classical RK4 steps with dt[m] (device,
 * FP64, per mesh).  When sample_every > 0, before every step whose index since the last
 * fr_reset_accumulators is a multiple of sample_every, the probe pressures (and wall forces
 * when enabled) of the current state are accumulated in FP64.  The step sequence is
 * replayed from a captured HIP graph. */
fr_status fr_rk_step(fr_solver *s, void *u, const double *dt, int32_t n_steps, int32_t sample_every,
                     void *stream);

/* Synchronise, then per probe (host out arrays, nullable): prms[a] = RMS of the sampled
 * pressure about its mean (Eqs. (10)-(12): last element of the cumulative vector),
 * oaspl[a] = 20 log10(prms / p_ref) (Eq. (9); -inf when prms = 0), mean_force[m*dim + j] =
 * time-mean wall force of mesh m, n_samples = samples taken.  FR_ERR_NONFINITE if a
 * sampled pressure is not finite. */
fr_status fr_probe_oaspl(fr_solver *s, double p_ref, double *prms, double *oaspl, double *mean_force,
                         int64_t *n_samples, void *stream);

/* Force coefficients of Eq. (8) (cavity drag; the airfoil's lift and drag): synchronise, then
 * coef[m*n_dir + k] = (time-mean wall force of mesh m) . dirs[(m*n_dir + k)*dim ...]
 *                     / (1/2 rho_inf,m |U_inf,m|^2 ref_area[m])
 * for n_dir caller-chosen directions per mesh (host arrays: dirs [n_mesh][n_dir][dim], unit
 * vectors, e.g. along and normal to the free stream; ref_area [n_mesh], e.g. chord x span; coef
 * [n_mesh][n_dir]).  The mean force is the FP64 sum of fr_probe_oaspl's mean_force.  FR_ERR_ARG
 * when the solver accumulates no forces, no sample was taken since the last reset, or an area or
 * free-stream dynamic pressure is not positive. */
fr_status fr_force_coefficients(fr_solver *s, int32_t n_dir, const double *dirs, const double *ref_area,
                                double *coef, void *stream);

/* Synchronise and copy the FP64 pressure series series[a*cap + k] for k < min(n, cap, max_samples);
 * *n = samples taken since the last reset (the device keeps the first max_samples of them). */
fr_status fr_probe_series(fr_solver *s, double *series, int64_t cap, int64_t *n, void *stream);

/* Zero the sample counter, probe sums / series and force sums (kernel fill, graph safe). */
fr_status fr_reset_accumulators(fr_solver *s, void *stream);

/* Vector-Jacobian product of fr_rhs (the adjoint of the residual at state u):
 * u_bar += (dR/du)^T r_bar.  u, r_bar, u_bar: device state arrays of the solver's dtype;
 * u_bar may not alias u or r_bar.  Overwrites the solver's flux-point work arrays (later
 * fr_rhs / fr_rk_step calls recompute them); allocates an adjoint work area on first use.
 * x_bar: NULL, or device FP64 [n_node][dim] that receives += (dR/dX)^T r_bar, the sensitivity to
 * the mesh node coordinates X through the metric terms (S = adj(dx/dxi), 1/J, Eq. (1) in
 * transformed form) and the face normals; with x_bar the call also evaluates the residual at u
 * and allocates the geometric adjoint tables on first use. */
fr_status fr_rhs_vjp(fr_solver *s, const void *u, const void *r_bar, void *u_bar, double *x_bar, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): fr_rhs_vjp without x_bar, u_bar += (dR/du)^T r_bar,
 * with the same kernels and the same result, whose work area (n_elem * nv * (Ns + 5 Nf) values
 * of the state dtype) is a library-owned static device buffer of FR_NOALLOC_SCRATCH_BYTES per
 * GPU instead of a per-solver allocation made on first use.  Allocates and frees nothing.  The
 * buffer is shared by every call on one GPU and keeps the last call's contents (every value is
 * written before it is read): calls that overlap in time on one GPU (other streams, other host
 * threads) race and must be ordered by the caller.  FR_ERR_ARG, before any launch, when the
 * solver's work area exceeds the buffer (the message gives both sizes) or on NULL / aliased
 * arguments.  Leaves the solver's forward work arrays untouched. */
#define FR_NOALLOC_SCRATCH_BYTES (32u << 20)
fr_status fr_rhs_vjp_noalloc(fr_solver *s, const void *u, const void *r_bar, void *u_bar, void *stream);

/* Counts of the discretisation: info[0..7] = {n_elem, nv, Ns, Nf, n_face_pairs (interior and
 * periodic flux-point pairs), n_boundary_points, n_wall_points, n_mesh}. */
fr_status fr_solver_info(const fr_solver *s, int64_t info[8]);

/* Kernel identifiers used by the timing interface. */
#define FR_K_INTERP      0   /* solution -> flux points                         */
#define FR_K_COMMON_SOL  1   /* LDG common solution (NS)                        */
#define FR_K_NS_GRAD     2   /* corrected gradient + fluxes + volume divergence */
#define FR_K_FACE_FLUX   3   /* common normal flux at every flux point          */
#define FR_K_DIV_RK      4   /* lifting + RK4 stage update + next u_f (NS)      */
#define FR_K_EULER_VOL   5   /* fluxes + divergence + RK4 update + next u_f     */
#define FR_K_PROBE       6   /* FP64 probe accumulator                          */
#define FR_K_FORCE       7   /* FP64 wall-force accumulator                     */
#define FR_K_COUNT       8

/* Per-kernel timing with HIP events recorded on the launch stream around every kernel.  While
 * enabled, fr_rhs / fr_rk_step launch kernels directly (no graph replay).  fr_profile_read
 * synchronises `stream` and returns, per kernel id, the summed duration in ms and the number of
 * launches since the last read (then resets them).  Arrays have FR_K_COUNT entries. */
fr_status fr_profile_enable(fr_solver *s, int32_t enable);
fr_status fr_profile_read(fr_solver *s, double *total_ms, int64_t *launches, void *stream);

/* Adjoint of the probe samples: u_bar += sum_a p_bar[a] dp_a/du with p_a the probe pressure
 * (interpolated conserved state, then Eq. (5)).  p_bar: device FP64 [n_probe].  x_bar: NULL, or
 * device FP64 [n_node][dim] += sum_a p_bar[a] dp_a/dX: the probe is fixed in physical space, so
 * its reference coordinates follow the nodes of its element. */
fr_status fr_probe_vjp(fr_solver *s, const void *u, const double *p_bar, void *u_bar, double *x_bar, void *stream);

/* n_steps classical RK4 steps of u (device state, in place, no sampling) that also store, for
 * every step n, the base state u_n in states[n][n_elem][nv][Ns] (skipped when states is NULL),
 * the three intermediate stage states y2 = u_n + dt/2 k1, y3 = u_n + dt/2 k2, y4 = u_n + dt k3 in
 * stages[n][3][n_elem][nv][Ns], and (skipped when residuals is NULL) the four stage residuals
 * k1..k4 in residuals[n][4][n_elem][nv][Ns] (device, state dtype), for use by fr_rk_step_vjp.
 * states and residuals must not alias u.  FR_ERR_ARG for n_steps < 1 or NULL u / dt / stages. */
fr_status fr_rk_step_stages(fr_solver *s, void *u, const double *dt, int32_t n_steps, void *states, void *stages,
                            void *residuals, void *stream);

/* Adjoint of one RK4 step u_n -> u_{n+1}: on entry u_bar holds dJ/du_{n+1}, on return dJ/du_n
 * (= (du_{n+1}/du_n)^T u_bar).  stages: the step's stage states from fr_rk_step_stages, or NULL
 * to recompute them from u_n.  dt: device FP64 [n_mesh].  x_bar: NULL, or device FP64
 * [n_node][dim] += (du_{n+1}/dX)^T u_bar (entry value of u_bar) through the residuals of the
 * four stages; residuals: the step's stage residuals from fr_rk_step_stages (used with x_bar),
 * or NULL to evaluate them.  Allocates its work area on first use. */
fr_status fr_rk_step_vjp(fr_solver *s, const void *u_n, const double *dt, const void *stages, const void *residuals,
                         void *u_bar, double *x_bar, void *stream);

/* Reverse of n_steps consecutive RK4 steps with their probe samples, the inner loop of a
 * checkpointed trajectory adjoint in one call: for j = n_steps-1 .. 0,
 *   u_bar <- (d u_{j+1} / d u_j)^T u_bar     (as fr_rk_step_vjp with states[j], stages[j]) and
 *   u_bar += sum_a p_bar[j][a] d p_a / d u_j (as fr_probe_vjp with states[j]).
 * states [n_steps][Ne][NV][Ns] (each step's base state), stages [n_steps][3][Ne][NV][Ns] and
 * residuals [n_steps][4][Ne][NV][Ns] (nullable; required with x_bar) as written by
 * fr_rk_step_stages; p_bar [n_steps][n_probe] FP64 (device); dt one device double per mesh.
 * x_bar (FP64 [n_node][dim], nullable): the mesh-node adjoint, only inside fr_geo_adjoint_begin /
 * _end (FR_ERR_ARG otherwise).  The sequence is captured into a HIP graph on first use and
 * replayed while the pointer arguments and n_steps repeat (a few such graphs are kept); the
 * solver's adjoint work areas are allocated on first use, before any capture.  u_bar must not
 * alias the inputs. */
fr_status fr_rk_segment_vjp(fr_solver *s, const void *states, const double *dt, const void *stages,
                            const void *residuals, const double *p_bar, int32_t n_steps, void *u_bar, double *x_bar,
                            void *stream);

/* Deferred mesh-node adjoint for reverse sweeps over many steps (the node mapping is linear, so
 * it can run once): after fr_geo_adjoint_begin, fr_rk_step_vjp calls with a non-NULL x_bar add
 * their metric and normal adjoints to the handle's accumulators without touching x_bar (their
 * probe terms, through fr_probe_vjp, still go to x_bar directly); fr_geo_adjoint_end maps the
 * accumulated adjoints to the nodes, x_bar (device FP64 [n_node][dim]) +=, and ends the mode.
 * fr_rhs_vjp with x_bar is refused (FR_ERR_ARG) while the mode is on. */
fr_status fr_geo_adjoint_begin(fr_solver *s, void *stream);
fr_status fr_geo_adjoint_end(fr_solver *s, double *x_bar, void *stream);

/* Autotuner.  For each volume kernel of the solver's equations (kind 0: NS volume kernel, 1: NS
 * lifting + RK kernel, 2: Euler volume + RK kernel, 3: NS volume adjoint kernel) the candidates
 * are the tile sizes (elements per workgroup: the default, its half and its quarter) times two
 * register budgets (the default and one alternative waves-per-SIMD launch bound), and for kind 0
 * in FP32 3-D p = 4 the volume divergence on the matrix cores; kind 3: default tile, half tile,
 * default tile with a launch bound; degree-0 groups have the default only.  kinds_mask: bit k
 * selects kind k (0: every kind of the solver's equations); the others keep their candidate and
 * report zero times.  fr_autotune times
 * each candidate on device copies of u (u is not modified) -- `reps` RK4 steps, or for kind 3
 * 4 x reps residual adjoints --, keeps the fastest, remembers it for the rest of the process under
 * (dim, p, precision, equations, LDG form, kind, floor(log2 n_elem)) -- a later solver with the
 * same key takes the remembered choice without timing -- and drops the captured step graphs so
 * that the next fr_rk_step re-captures them.  Synchronises `stream`; allocates and frees
 * state-sized scratch copies (and the adjoint's work area) when it times.
 * choice[4][4] (host, nullable): per kind (elements per workgroup, waves-per-SIMD bound or 0 for
 * the compiler's default, engine 0 vector ALU / 1 matrix cores, 1 if taken from the remembered
 * choices; zeros for kinds the solver does not run).  ms[4][FR_TUNE_MAX] (host, nullable): ms per
 * RK4 step (kind 3: per 4 residual adjoints) of each candidate, 0 where not timed.  FR_ERR_ARG for
 * reps < 1.
 * fr_tune_candidates: the candidates of `kind`, cand[FR_TUNE_MAX][3] as in choice, *n of them.
 * fr_tune_select: use candidate `index` of `kind` from now on (drops the step graphs).
 * fr_tune_cache_clear: forget the remembered choices. */
#define FR_TUNE_MAX 8
fr_status fr_autotune(fr_solver *s, const void *u, const double *dt, int32_t reps, int32_t kinds_mask,
                      int32_t *choice, double *ms, void *stream);
fr_status fr_tune_candidates(const fr_solver *s, int32_t kind, int32_t *cand, int32_t *n);
fr_status fr_tune_select(fr_solver *s, int32_t kind, int32_t index);
void fr_tune_cache_clear(void);

/* Host statistics of FP64 probe pressure series (no solver, no device; plain host arrays).
 *
 * fr_stats_prms_cumulative: the vectors of Eqs. (10)-(12): prms[k] (k < n) is the RMS of the
 * first k+1 samples about their own mean (the cumulative time average); prms[n-1] is the p_RMS
 * of Eq. (9).  FR_ERR_ARG for NULL or n < 1.
 *
 * fr_stats_observer_oaspl: several observer points per observer (the spanwise probes of one
 * observer location): series[a][n] for probes a < n_probe, group[a] in [0, n_group) the observer
 * of probe a.  Per observer g: prms[g] = mean over its probes of each probe's p_RMS (Eq. (9)),
 * oaspl[g] = 20 log10(prms[g] / p_ref).  FR_ERR_ARG for bad sizes, a group without probes or
 * p_ref <= 0.
 *
 * fr_stats_psd_welch: Welch's method of averaged periodograms for the pressure perturbation:
 * n_windows segments of even length L = 2 floor(n / (n_windows + 1)) with 50% overlap, each
 * demeaned and multiplied by the periodic Hann window; one-sided density
 * psd[f] = c_f sum over segments |DFT|^2 / (n_windows fs sum w^2) (c_f = 2 except at 0 and fs/2),
 * freq[f] = f fs / L for f = 0..L/2, fs = 1 / sample_dt.  *n_freq = L/2 + 1; FR_ERR_ARG when cap
 * is smaller, n_windows < 1, sample_dt <= 0 or the series is too short. */
fr_status fr_stats_prms_cumulative(const double *series, int64_t n, double *prms);
fr_status fr_stats_observer_oaspl(const double *series, int32_t n_probe, int64_t n, const int32_t *group,
                                  int32_t n_group, double p_ref, double *prms, double *oaspl);
fr_status fr_stats_psd_welch(const double *series, int64_t n, int32_t n_windows, double sample_dt, double *freq,
                             double *psd, int64_t cap, int64_t *n_freq);

/* Release everything the handle owns (NULL is a no-op). */
void fr_destroy(fr_solver *s);

/*
 * Variable solution degree (the sponge of the airfoil case's computational details: the
 * degree falls from 4 or 3 near the airfoil to 0 towards the outer boundaries so that outgoing
 * waves are damped before they reach them).  The paper gives the distribution, not the face
 * treatment; the one built here:
 *  - every element is FR of its own degree p_e in 0..4 (Gauss-Legendre points, g_DG
 *    correction; degree 0 is one point with correction derivative 1/2: a finite-volume cell);
 *  - faces between equal degrees are treated as in fr_build_operators;
 *  - a face between degrees p_lo < p_hi is a mortar on the higher side's flux points: the lower
 *    side's trace polynomial is evaluated there, the LDG common solution and the common flux
 *    (Rusanov + LDG with each side's own viscous normal flux carried to the mortar, penalty
 *    tau) are formed there with the higher side's normal and |N|; the higher side takes them at
 *    its own points, the lower side their L2 projections onto its face polynomials (Gauss
 *    quadrature on the mortar points), so each face's integrated flux is the same from both
 *    sides (conservative).  Free-stream preserving where the face normal is a polynomial of
 *    degree <= p_lo along the face (faces along z of an extruded mesh with in-plane degrees).
 * Restrictions: Navier-Stokes, one mesh (n_mesh <= 1), probes in that mesh; the adjoint entry
 * points take single-degree solvers only.
 *
 * fr_vdeg_build: mesh as for fr_build_operators (its p is ignored); elem_degree[n_elem] in
 *   0..4 (host, read during the call); params as for fr_build_operators.  FR_ERR_UNSUPPORTED
 *   for Euler or several meshes, FR_ERR_MESH for a face between degrees that is not conforming.
 * State layout (device, precision of params): one buffer holding the degree groups in
 *   increasing degree; group g starts at value offset[g] and is [n_elem[g]][dim+2][(degree+1)^dim]
 *   with its elements in increasing element number (fr_vdeg_group_elems); offset[n_group] is the
 *   buffer length in values (each group starts on a 64-value boundary; the gaps are not read).
 * fr_vdeg_groups: n_group, degree[g] (-1 past n_group), n_elem[g], offset[0..5], and the number
 *   of mortar faces.  fr_vdeg_solpt_coords: xyz[n_elem[g]][(degree+1)^dim][dim] of group g.
 * fr_vdeg_rhs / fr_vdeg_rk_step / fr_vdeg_reset_accumulators: as fr_rhs / fr_rk_step /
 *   fr_reset_accumulators on the whole buffer (u and r must not alias; dt is one device double).
 * fr_vdeg_probe_series: as fr_probe_series, probes in the order given at build.
 * fr_vdeg_mean_force: mean wall force [dim] over the samples since the last reset (forces != 0),
 *   *n_samples the number of samples; FR_ERR_NONFINITE if a sampled probe pressure was not finite.
 */
typedef struct fr_vdeg fr_vdeg;  /* opaque, library-owned */
fr_status fr_vdeg_build(const fr_mesh_desc *mesh, const int32_t *elem_degree, const fr_params *params,
                        fr_vdeg **out);
fr_status fr_vdeg_groups(const fr_vdeg *v, int32_t *n_group, int32_t degree[5], int64_t n_elem[5],
                         int64_t offset[6], int64_t *n_mortar);
fr_status fr_vdeg_group_elems(const fr_vdeg *v, int32_t group, int64_t *elems);
fr_status fr_vdeg_solpt_coords(const fr_vdeg *v, int32_t group, double *xyz);
fr_status fr_vdeg_rhs(fr_vdeg *v, const void *u, void *r, void *stream);
fr_status fr_vdeg_rk_step(fr_vdeg *v, void *u, const double *dt, int32_t n_steps, int32_t sample_every,
                          void *stream);
fr_status fr_vdeg_reset_accumulators(fr_vdeg *v, void *stream);
fr_status fr_vdeg_probe_series(fr_vdeg *v, double *series, int64_t cap, int64_t *n, void *stream);
fr_status fr_vdeg_mean_force(fr_vdeg *v, double *mean_force, int64_t *n_samples, void *stream);
void fr_vdeg_destroy(fr_vdeg *v);

/* Thread-local message of the last failing call ("" if none). */
const char *fr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FRMI_FR_H */
