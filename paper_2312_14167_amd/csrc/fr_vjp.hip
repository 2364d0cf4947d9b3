// Vector-Jacobian product of the FR residual: u_bar += (dR/du)^T r_bar, hand-derived, for the
// Euler and Navier-Stokes forms in 2-D and 3-D.  The residual (Eqs. (1)-(7) discretised by FR) is
//   R = -(1/J) [ vol + Lift F^ ],  vol = sum_k D_k F~_k - Lift (s_f M0 F~_{k_f}),
// with F~_k = S_k . (F_inv(u) - F_vis(u, grad u)) and F^ the common normal flux.  Its adjoint runs
// the pipeline backwards:
//   vjp_div    w = -(1/J) r_bar;  vol_bar = w;  F^_bar = Lift^T w                  (element local)
//   vjp_face   Rusanov / LDG / boundary adjoints -> u_f_bar (both sides), fvn_bar   (per flux point)
//   vjp_vol    recompute u_f, u^, grad u, F~ in LDS; F~_bar = (D_k - Lift s M0)^T vol_bar;
//              pointwise flux adjoints -> u_bar, grad_bar; fvn adjoint at flux points; transposed
//              corrected gradient -> u_bar, (u^ - u_f)_bar -> own / neighbour u_f_bar
//   vjp_final  u_bar += u_vol_bar + M0^T (u_f_bar own + neighbour)
// Kink conventions: |x| has derivative 0 at 0; max(a_L, a_R) of the Rusanov speed sends its
// adjoint to the larger side, and half to each side when the two agree to a relative 1e-12.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fr_device.hpp"
#include "fr_dispatch.hpp"

namespace frmi {

// ------------------------------------------------------------------------------------ pointwise adjoints
template <int D, typename T>
__device__ __forceinline__ void pressure_grad(const T *u, T gm1, T &p, T *dp) {
  const T r = T(1) / u[0];
  T m2 = T(0);
  for (int j = 0; j < D; ++j) m2 += u[1 + j] * u[1 + j];
  p = gm1 * (u[D + 1] - T(0.5) * m2 * r);
  dp[0] = gm1 * T(0.5) * m2 * r * r;
  for (int j = 0; j < D; ++j) dp[1 + j] = -gm1 * u[1 + j] * r;
  dp[D + 1] = gm1;
}

// ub += (d (F_inv(u) . m) / du)^T fb
template <int D, typename T>
__device__ __forceinline__ void finv_dot_vjp(const T *u, const T *m, T gm1, const T *fb, T *ub) {
  constexpr int NV = D + 2;
  T p, dp[NV];
  pressure_grad<D>(u, gm1, p, dp);
  const T r = T(1) / u[0];
  T a = T(0);
  for (int j = 0; j < D; ++j) a += u[1 + j] * m[j];
  const T ar = a * r, H = u[D + 1] + p;
  T Pb = fb[D + 1] * ar, q = T(0);
  for (int i = 0; i < D; ++i) {
    Pb += fb[1 + i] * m[i];
    q += fb[1 + i] * u[1 + i];
  }
  const T arb = q + fb[D + 1] * H;
  ub[0] += arb * (-a * r * r) + Pb * dp[0];
  for (int j = 0; j < D; ++j) ub[1 + j] += fb[0] * m[j] + fb[1 + j] * ar + arb * m[j] * r + Pb * dp[1 + j];
  ub[D + 1] += fb[D + 1] * ar + Pb * dp[D + 1];
}

// ub += ab * d(|v.n| + c)/du
template <int D, typename T>
__device__ __forceinline__ void wavespeed_vjp(const T *u, const T *n, T gamma, T gm1, T ab, T *ub) {
  constexpr int NV = D + 2;
  T p, dp[NV];
  pressure_grad<D>(u, gm1, p, dp);
  const T r = T(1) / u[0];
  T vn = T(0);
  for (int j = 0; j < D; ++j) vn += u[1 + j] * n[j];
  vn *= r;
  const T sg = vn > T(0) ? T(1) : (vn < T(0) ? T(-1) : T(0));
  const T c = sqrt(gamma * p * r);
  const T cf = ab * gamma / (T(2) * c);
  ub[0] += ab * sg * (-vn * r) + cf * (dp[0] * r - p * r * r);
  for (int j = 0; j < D; ++j) ub[1 + j] += ab * sg * n[j] * r + cf * dp[1 + j] * r;
  ub[D + 1] += cf * dp[D + 1] * r;
}

template <int D, typename T>
__device__ __forceinline__ T wavespeed(const T *u, const T *n, T gamma, T gm1) {
  T rho, v[D], p;
  primitives<D>(u, gm1, rho, v, p);
  T vn = T(0);
  for (int j = 0; j < D; ++j) vn += v[j] * n[j];
  return fabs(vn) + sqrt(gamma * p / rho);
}

// adjoint of rusanov(): uLb += (dF/duL)^T Fb, uRb += (dF/duR)^T Fb
template <int D, typename T>
__device__ __forceinline__ void rusanov_vjp(const T *uL, const T *uR, const T *n, T gamma, T gm1, const T *Fb,
                                            T *uLb, T *uRb) {
  constexpr int NV = D + 2;
  T hb[NV];
  for (int v = 0; v < NV; ++v) hb[v] = T(0.5) * Fb[v];
  finv_dot_vjp<D>(uL, n, gm1, hb, uLb);
  finv_dot_vjp<D>(uR, n, gm1, hb, uRb);
  const T aL = wavespeed<D>(uL, n, gamma, gm1), aR = wavespeed<D>(uR, n, gamma, gm1);
  const T lam = aL >= aR ? aL : aR;
  T lamb = T(0);
  for (int v = 0; v < NV; ++v) {
    uLb[v] += T(0.5) * lam * Fb[v];
    uRb[v] -= T(0.5) * lam * Fb[v];
    lamb -= T(0.5) * Fb[v] * (uR[v] - uL[v]);
  }
  // max(aL, aR): the larger side, or half to each when they agree to a relative 1e-12 (FP64) /
  // 1e-5 (FP32), so that round-off cannot flip the side of the kink
  const T tol = (sizeof(T) == 8 ? T(1e-12) : T(1e-5)) * (aL >= aR ? aL : aR);
  if (aL - aR > tol)
    wavespeed_vjp<D>(uL, n, gamma, gm1, lamb, uLb);
  else if (aR - aL > tol)
    wavespeed_vjp<D>(uR, n, gamma, gm1, lamb, uRb);
  else {
    wavespeed_vjp<D>(uL, n, gamma, gm1, T(0.5) * lamb, uLb);
    wavespeed_vjp<D>(uR, n, gamma, gm1, T(0.5) * lamb, uRb);
  }
}

// adjoint of the viscous flux F_vis(st, g) . m with the conserved gradient g[d * NV + v]
template <int D, typename T>
__device__ __forceinline__ void fvis_vjp(const T *st, const T *g, const T *m, T mu, const PhysDev<T> &ph, bool heat,
                                         const T *fb, T *stb, T *gb) {
  constexpr int NV = D + 2;
  const T r = T(1) / st[0];
  const T Es = st[D + 1] * r;
  T vel[D], dv[D][D];
  for (int i = 0; i < D; ++i) vel[i] = st[1 + i] * r;
  for (int d = 0; d < D; ++d)
    for (int i = 0; i < D; ++i) dv[i][d] = (g[d * NV + 1 + i] - vel[i] * g[d * NV]) * r;
  T div = T(0);
  for (int i = 0; i < D; ++i) div += dv[i][i];
  const T c23 = T(2) / T(3);
  T tn[D];
  for (int i = 0; i < D; ++i) {
    T s = T(0);
    for (int d = 0; d < D; ++d) s += (dv[i][d] + dv[d][i]) * m[d];
    tn[i] = mu * (s - c23 * div * m[i]);
  }
  const T kappa = heat ? mu * ph.gamma / (ph.prandtl * ph.gm1) : T(0);
  T tb[D], vb[D];
  T tm = T(0);
  for (int i = 0; i < D; ++i) {
    tb[i] = fb[1 + i] + fb[D + 1] * vel[i];
    vb[i] = fb[D + 1] * tn[i];
    tm += tb[i] * m[i];
  }
  T rb = T(0), Esb = T(0);
  for (int d = 0; d < D; ++d) {
    // d_theta_d = gm1 ((g_dE - Es g_d0) r - sum_i v_i dv_id)
    const T x = fb[D + 1] * kappa * m[d] * ph.gm1;
    gb[d * NV + D + 1] += x * r;
    gb[d * NV] -= x * Es * r;
    Esb -= x * g[d * NV] * r;
    rb += x * (g[d * NV + D + 1] - Es * g[d * NV]);
    for (int i = 0; i < D; ++i) {
      // dv_id adjoint: stress part minus the heat-flux part
      const T y = mu * (tb[i] * m[d] + tb[d] * m[i] - (i == d ? c23 * tm : T(0))) - x * vel[i];
      vb[i] -= x * dv[i][d];
      gb[d * NV + 1 + i] += y * r;
      gb[d * NV] -= y * vel[i] * r;
      vb[i] -= y * g[d * NV] * r;
      rb += y * (g[d * NV + 1 + i] - vel[i] * g[d * NV]);
    }
  }
  for (int i = 0; i < D; ++i) {
    stb[1 + i] += vb[i] * r;
    rb += vb[i] * st[1 + i];
  }
  stb[D + 1] += Esb * r;
  rb += Esb * st[D + 1];
  stb[0] -= rb * r * r;
}

// adjoint of farfield(): uLb += (d ub / d uL)^T ubb
template <int D, typename T>
__device__ __forceinline__ void farfield_vjp(const T *uL, const T *n, const FlowDev<T> &fl, T gamma, T gm1,
                                             const T *ubb, T *uLb, T *nb = nullptr) {
  // forward recompute
  const T rL = uL[0];
  T vL[D], m2 = T(0);
  for (int j = 0; j < D; ++j) {
    vL[j] = uL[1 + j] / rL;
    m2 += uL[1 + j] * uL[1 + j];
  }
  const T pL = gm1 * (uL[D + 1] - T(0.5) * m2 / rL);
  const T cL = sqrt(gamma * pL / rL);
  const T ci = sqrt(gamma * fl.p / fl.rho);
  T vnL = T(0), vni = T(0);
  for (int j = 0; j < D; ++j) { vnL += vL[j] * n[j]; vni += fl.v[j] * n[j]; }
  const T Rp = vnL + T(2) * cL / gm1;
  const T Rm = vni - T(2) * ci / gm1;
  const T vn = T(0.5) * (Rp + Rm);
  const T c = T(0.25) * gm1 * (Rp - Rm);
  const bool out = vn > T(0);
  const T s = out ? pL / pow(rL, gamma) : fl.p / pow(fl.rho, gamma);
  const T X = c * c / (gamma * s);
  const T rho = pow(X, T(1) / gm1);
  T v[D], v2 = T(0);
  for (int j = 0; j < D; ++j) {
    const T vt = out ? vL[j] - vnL * n[j] : fl.v[j] - vni * n[j];
    v[j] = vt + vn * n[j];
    v2 += v[j] * v[j];
  }
  // reverse
  T rhob = ubb[0] + T(0.5) * v2 * ubb[D + 1];
  T vb[D];
  for (int j = 0; j < D; ++j) {
    rhob += ubb[1 + j] * v[j];
    vb[j] = ubb[1 + j] * rho + ubb[D + 1] * rho * v[j];
  }
  const T pb = ubb[D + 1] / gm1;
  rhob += pb * c * c / gamma;
  T cb = pb * T(2) * rho * c / gamma;
  const T Xb = rhob * rho / (gm1 * X);
  cb += Xb * T(2) * c / (gamma * s);
  const T sb = -Xb * X / s;
  T vnb = T(0);
  for (int j = 0; j < D; ++j) vnb += vb[j] * n[j];
  if (nb) {
    // n enters through v = w + (vn - vn_w) n (w = v_L or v_inf by the branch), vn and c; the
    // branch itself (sign of vn) is piecewise constant
    const T vnw = out ? vnL : vni;
    for (int m = 0; m < D; ++m) {
      const T dvn = T(0.5) * (vL[m] + fl.v[m]), dc = T(0.25) * gm1 * (vL[m] - fl.v[m]);
      const T dvw = out ? vL[m] : fl.v[m];
      nb[m] += (dvn - dvw) * vnb + (vn - vnw) * vb[m] + cb * dc;
    }
  }
  const T Rpb = T(0.5) * vnb + T(0.25) * gm1 * cb;
  T vnLb = Rpb;
  T cLb = T(2) * Rpb / gm1;
  T vLb[D];
  T pLb = T(0), rLb = T(0);
  for (int j = 0; j < D; ++j) vLb[j] = T(0);
  if (out) {
    T tdot = T(0);
    for (int j = 0; j < D; ++j) {
      vLb[j] += vb[j];
      tdot += vb[j] * n[j];
    }
    vnLb -= tdot;
    const T rg = pow(rL, gamma);
    pLb += sb / rg;
    rLb -= gamma * sb * pL / (rg * rL);
  }
  for (int j = 0; j < D; ++j) vLb[j] += vnLb * n[j];
  pLb += cLb * gamma / (T(2) * cL * rL);
  rLb -= cLb * gamma * pL / (T(2) * cL * rL * rL);
  for (int j = 0; j < D; ++j) {
    uLb[1 + j] += vLb[j] / rL - gm1 * pLb * uL[1 + j] / rL;
    rLb -= vLb[j] * uL[1 + j] / (rL * rL);
  }
  uLb[D + 1] += gm1 * pLb;
  rLb += gm1 * pLb * T(0.5) * m2 / (rL * rL);
  uLb[0] += rLb;
}

// adjoint of wall_state() (zero velocity, same density and internal energy)
template <int D, typename T>
__device__ __forceinline__ void wall_state_vjp(const T *uB, const T *wb, T *uBb) {
  const T r = T(1) / uB[0];
  T m2 = T(0);
  for (int j = 0; j < D; ++j) m2 += uB[1 + j] * uB[1 + j];
  uBb[0] += wb[0] + wb[D + 1] * T(0.5) * m2 * r * r;
  for (int j = 0; j < D; ++j) uBb[1 + j] -= wb[D + 1] * uB[1 + j] * r;
  uBb[D + 1] += wb[D + 1];
}

// row k of a small matrix without dynamic indexing into a private array (k is a loop counter of
// a loop the compiler keeps rolled)
template <int D, typename T>
__device__ __forceinline__ void pick_row(const T (&M)[D][D], int k, T (&r)[D]) {
  for (int j = 0; j < D; ++j) {
    r[j] = M[0][j];
    for (int q = 1; q < D; ++q)
      if (k == q) r[j] = M[q][j];
  }
}

// ------------------------------------------------------------------------------------ geometric adjoints
// nb += d(Fb . rusanov(uL, uR, n)) / dn with the states held fixed (the wave-speed max follows
// the tie rule of rusanov_vjp)
template <int D, typename T>
__device__ __forceinline__ void rusanov_n_vjp(const T *uL, const T *uR, const T *n, T gamma, T gm1, const T *Fb,
                                              T *nb) {
  constexpr int NV = D + 2;
  T rL, vL[D], pL, rR, vR[D], pR;
  primitives<D>(uL, gm1, rL, vL, pL);
  primitives<D>(uR, gm1, rR, vR, pR);
  // 1/2 (F_inv(uL) + F_inv(uR)) . n: column j dotted with Fb
  for (int j = 0; j < D; ++j) {
    T s = Fb[0] * (uL[1 + j] + uR[1 + j]) + Fb[D + 1] * (vL[j] * (uL[D + 1] + pL) + vR[j] * (uR[D + 1] + pR));
    for (int i = 0; i < D; ++i) s += Fb[1 + i] * (uL[1 + i] * vL[j] + uR[1 + i] * vR[j]);
    s += Fb[1 + j] * (pL + pR);
    nb[j] += T(0.5) * s;
  }
  T vnL = T(0), vnR = T(0), lamb = T(0);
  for (int j = 0; j < D; ++j) { vnL += vL[j] * n[j]; vnR += vR[j] * n[j]; }
  for (int v = 0; v < NV; ++v) lamb -= T(0.5) * Fb[v] * (uR[v] - uL[v]);
  const T aL = fabs(vnL) + sqrt(gamma * pL / rL), aR = fabs(vnR) + sqrt(gamma * pR / rR);
  const T tol = (sizeof(T) == 8 ? T(1e-12) : T(1e-5)) * (aL >= aR ? aL : aR);
  const T wL = aL - aR > tol ? T(1) : (aR - aL > tol ? T(0) : T(0.5));
  const T sL = vnL > T(0) ? T(1) : (vnL < T(0) ? T(-1) : T(0));
  const T sR = vnR > T(0) ? T(1) : (vnR < T(0) ? T(-1) : T(0));
  for (int j = 0; j < D; ++j) nb[j] += lamb * (wL * sL * vL[j] + (T(1) - wL) * sR * vR[j]);
}

// out[j] += sum_v w[v] F_vis,j[v] (viscous flux column j, from the viscous state vs)
template <int D, typename T>
__device__ __forceinline__ void fvis_columns_dot(const Visc<D, T> &vs, const T *w, T *out) {
  for (int j = 0; j < D; ++j) {
    T s = T(0), en = T(0);
    for (int i = 0; i < D; ++i) {
      s += w[1 + i] * vs.tau[i][j];
      en += vs.v[i] * vs.tau[i][j];
    }
    out[j] += s + w[D + 1] * (en - vs.q[j]);
  }
}

// out[j] += sum_v w[v] F_inv,j[v] (inviscid flux column j)
template <int D, typename T>
__device__ __forceinline__ void finv_columns_dot(const T *u, T gm1, const T *w, T *out) {
  T rho, v[D], p;
  primitives<D>(u, gm1, rho, v, p);
  for (int j = 0; j < D; ++j) {
    T s = w[0] * u[1 + j] + w[D + 1] * v[j] * (u[D + 1] + p) + w[1 + j] * p;
    for (int i = 0; i < D; ++i) s += w[1 + i] * u[1 + i] * v[j];
    out[j] += s;
  }
}

// A = adj(S) (1/J)^(D-2) from the stored metric (S = adj(A)), A[j][k] = dx_j/dxi_k
template <int D, typename T>
__device__ __forceinline__ void jacobian_from_metric(const T (&Sm)[D][D], T invJ, T (&A)[D][D]) {
  if (D == 2) {
    A[0][0] = Sm[1][1];
    A[0][1] = -Sm[0][1];
    A[1][0] = -Sm[1][0];
    A[1][1] = Sm[0][0];
  } else {
    for (int r = 0; r < D; ++r) {
      const int a = (r + 1) % D, b = (r + 2) % D;  // row r of adj(S) = column a x column b of S
      A[r][0] = (Sm[1][a] * Sm[2][b] - Sm[2][a] * Sm[1][b]) * invJ;
      A[r][1] = (Sm[2][a] * Sm[0][b] - Sm[0][a] * Sm[2][b]) * invJ;
      A[r][2] = (Sm[0][a] * Sm[1][b] - Sm[1][a] * Sm[0][b]) * invJ;
    }
  }
}

// ------------------------------------------------------------------------------------ kernels
template <int D, int P, typename T>
struct VjpDivTile {
  using S = Shape<D, P>;
  static constexpr int LE = S::NV * S::Ns;
  static constexpr int E = tile_elems<S::Ns>(LE, sizeof(T));
  static constexpr int BS = round64(E * S::Ns);
};

// w = -(1/J) r_bar -> vol_bar (solution points) and F^_bar = Lift^T w (flux points); also the
// forward flux-point values u_f = M0 u at the linearisation point (read by the face adjoint)
// GEO: also the adjoint of 1/J, r_bar . R / (1/J) (R the forward residual), into Gm
// RKIN (first reverse stage of an RK4 step): rbar is the step's entry adjoint a, r_bar = dt ca a
// is formed here and a is copied to rk_a (read by every stage's epilogue)
template <int D, int P, typename T, bool GEO, bool RKIN = false>
__global__ __launch_bounds__((VjpDivTile<D, P, T>::BS)) void k_vjp_div(const T *__restrict__ rbar,
                                                                       const T *__restrict__ u,
                                                                       const T *__restrict__ metric,
                                                                       OpsDev<T, P> ops_arg, T *__restrict__ volbar,
                                                                       T *__restrict__ fhatbar, T *__restrict__ uf,
                                                                       const T *__restrict__ Rf, T *__restrict__ Gm,
                                                                       int64_t Ne, T *__restrict__ rk_a = nullptr,
                                                                       const double *__restrict__ dt = nullptr,
                                                                       const int32_t *__restrict__ elem_mesh = nullptr,
                                                                       T ca = T(0)) {
  using S = Shape<D, P>;
  using TL = VjpDivTile<D, P, T>;
  constexpr int E = TL::E, Ns = S::Ns, Nf = S::Nf, NV = S::NV, NM = S::NM;
  __shared__ __attribute__((aligned(16))) T lw[E * TL::LE];
  __shared__ __attribute__((aligned(16))) T lu[E * TL::LE];
  __shared__ OpsDev<T, P> ops;
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (int)((Ne - e0) < E ? (Ne - e0) : E);
  const int el = threadIdx.x / Ns, i = threadIdx.x % Ns;
  const int64_t e = e0 + el;
  // the state tile and this point's operands in one round trip
  TileLoad<E * NV * Ns, TL::BS, T> tu;
  tu.load(u + e0 * NV * Ns, ne * NV * Ns);
  T invJ = T(0), rb[NV], rf[NV], gprev = T(0), scale = T(1);
  if (el < ne) {
    invJ = metric[(e * NM + D * D) * Ns + i];
    for (int v = 0; v < NV; ++v) {
      rb[v] = rbar[(e * NV + v) * Ns + i];
      if (GEO) rf[v] = Rf[(e * NV + v) * Ns + i];
    }
    if (GEO) gprev = Gm[(e * NM + D * D) * Ns + i];
    if (RKIN) scale = (T)dt[elem_mesh[e]] * ca;
  }
  stage_ops(ops, ops_arg);
  tu.store(lu, ne * NV * Ns);
  if (el < ne) {
    if (RKIN)
      for (int v = 0; v < NV; ++v) {
        rk_a[(e * NV + v) * Ns + i] = rb[v];
        rb[v] *= scale;
      }
    T gj = T(0);
    for (int v = 0; v < NV; ++v) {
      const T w = -invJ * rb[v];
      lw[(el * NV + v) * Ns + i] = w;
      volbar[(e * NV + v) * Ns + i] = w;
      if (GEO) gj += rb[v] * rf[v];
    }
    if (GEO) Gm[(e * NM + D * D) * Ns + i] = gprev + gj / invJ;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < ne * NV * Nf; idx += blockDim.x) {
    const int fp = idx % Nf, rest = idx / Nf;
    int base, stride, side;
    line_of_fpt<D, P>(fp, base, stride, side);
    const T *g = side ? ops.gp : ops.gm;
    const T *lv = side ? ops.lp : ops.lm;
    const T *lin = lw + rest * Ns + base;
    const T *lun = lu + rest * Ns + base;
    T s = T(0), su = T(0);
#pragma unroll
    for (int a = 0; a < P; ++a) {
      s += g[a] * lin[a * stride];
      su += lv[a] * lun[a * stride];
    }
    fhatbar[e0 * NV * Nf + idx] = s;
    uf[e0 * NV * Nf + idx] = su;
  }
}

// Adjoint of one interior pair's common flux F^ |N| = [Rusanov(u_L, u_R, n) + tau (u_L - u_R)
// - viscous share] |N| (written with + on the L side, - on the R side): from the common-flux
// adjoints of both sides, the u_f adjoints of both sides and (NS) the adjoints of each side's
// viscous normal flux.  GEO: the adjoint of the unit normal (nb, +=) and of |N| (mb, =).
template <int D, typename T, bool NS, bool GEO>
__device__ __forceinline__ void pair_flux_vjp(const T *uL, const T *uR, const T *n, T mag, const T *fhbL,
                                              const T *fhbR, const PhysDev<T> &ph, T *uLb, T *uRb, T *fvbL,
                                              T *fvbR, T *nb, T &mb) {
  constexpr int NV = D + 2;
  T Fb[NV];
  for (int v = 0; v < NV; ++v) {
    Fb[v] = mag * (fhbL[v] - fhbR[v]);
    uLb[v] = T(0);
    uRb[v] = T(0);
  }
  rusanov_vjp<D>(uL, uR, n, ph.gamma, ph.gm1, Fb, uLb, uRb);
  if (GEO) {
    // |N|_bar = sum (F^_bar_L - F^_bar_R) . F with F = Rusanov + penalty - viscous part; the
    // viscous part is added by the volume adjoint, which recomputes each side's fvn
    T Fr[NV];
    rusanov_n_vjp<D>(uL, uR, n, ph.gamma, ph.gm1, Fb, nb);
    rusanov<D>(uL, uR, n, ph.gamma, ph.gm1, Fr);
    mb = T(0);
    for (int v = 0; v < NV; ++v) mb += Fb[v] * (Fr[v] + (NS ? ph.tau * (uL[v] - uR[v]) : T(0)));
  }
  if (NS) {
    const T wl = T(0.5) - ph.beta, wr = T(0.5) + ph.beta;
    for (int v = 0; v < NV; ++v) {
      uLb[v] += ph.tau * Fb[v];
      uRb[v] -= ph.tau * Fb[v];
      fvbL[v] = -wl * Fb[v];
      fvbR[v] = wr * Fb[v];
    }
  }
}

// Adjoint of a boundary point's common flux (Rusanov against the wall reflection or the far-field
// state, minus the viscous normal flux): u_f adjoint and (NS) the viscous-normal-flux adjoint.
template <int D, typename T, bool NS, bool GEO>
__device__ __forceinline__ void bnd_flux_vjp(const T *uB, const T *n, T mag, const T *fhb, bool wall,
                                             const FlowDev<T> &fl, const PhysDev<T> &ph, T *uBb, T *fvb, T *nb,
                                             T &mb) {
  constexpr int NV = D + 2;
  T ug[NV], Fb[NV], ugb[NV];
  for (int v = 0; v < NV; ++v) {
    Fb[v] = mag * fhb[v];
    uBb[v] = T(0);
    ugb[v] = T(0);
  }
  if (wall) {
    ug[0] = uB[0];
    for (int j = 0; j < D; ++j) ug[1 + j] = -uB[1 + j];
    ug[D + 1] = uB[D + 1];
  } else {
    farfield<D>(uB, n, fl, ph.gamma, ph.gm1, ug);
  }
  rusanov_vjp<D>(uB, ug, n, ph.gamma, ph.gm1, Fb, uBb, ugb);
  if (GEO) rusanov_n_vjp<D>(uB, ug, n, ph.gamma, ph.gm1, Fb, nb);
  if (wall) {
    uBb[0] += ugb[0];
    for (int j = 0; j < D; ++j) uBb[1 + j] -= ugb[1 + j];
    uBb[D + 1] += ugb[D + 1];
  } else {
    farfield_vjp<D>(uB, n, fl, ph.gamma, ph.gm1, ugb, uBb, GEO ? nb : nullptr);
  }
  if (GEO) {
    T Fr[NV];
    rusanov<D>(uB, ug, n, ph.gamma, ph.gm1, Fr);
    mb = T(0);
    for (int v = 0; v < NV; ++v) mb += Fb[v] * Fr[v];
  }
  if (NS)
    for (int v = 0; v < NV; ++v) fvb[v] = -Fb[v];
}

// adjoint of the common-flux kernel, one thread per pair or boundary point: u_f_bar of both sides
// and (NS) the viscous-normal-flux adjoints.  (The Navier-Stokes volume adjoint forms the same
// per side itself; this kernel serves the Euler path.)
// GEO: also the adjoints of the unit normal (Rusanov, far-field ghost) and the inviscid and
// penalty part of the adjoint of |N| at the owning point (L side / boundary point), into Gn
template <int D, int P, typename T, bool NS, bool GEO>
__global__ __launch_bounds__(256) void k_vjp_face(const T *__restrict__ uf, const T *__restrict__ fhatbar,
                                                  const int32_t *__restrict__ pairL, const int32_t *__restrict__ pairR,
                                                  const T *__restrict__ pnrm, int64_t npair,
                                                  const int32_t *__restrict__ bnd, const T *__restrict__ bnrm,
                                                  int64_t n_wall, int64_t nbnd, const int32_t *__restrict__ elem_mesh,
                                                  const FlowDev<T> *__restrict__ flow, PhysDev<T> ph,
                                                  T *__restrict__ ufbar, T *__restrict__ fvnbar,
                                                  T *__restrict__ Gn) {
  using S = Shape<D, P>;
  constexpr int NV = S::NV, Nf = S::Nf;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < npair) {
    const int32_t cL = pairL[gid], cR = pairR[gid];
    const int64_t eL = cL / Nf, eR = cR / Nf;
    const int fL = cL % Nf, fR = cR % Nf;
    T uL[NV], uR[NV], n[D], fhL[NV], fhR[NV], uLb[NV], uRb[NV], fvL[NV], fvR[NV], nb[D], mb = T(0);
    for (int j = 0; j < D; ++j) {
      n[j] = pnrm[gid * (D + 1) + j];
      nb[j] = T(0);
    }
    const T mag = pnrm[gid * (D + 1) + D];
    for (int v = 0; v < NV; ++v) {
      uL[v] = uf[(eL * NV + v) * Nf + fL];
      uR[v] = uf[(eR * NV + v) * Nf + fR];
      fhL[v] = fhatbar[(eL * NV + v) * Nf + fL];
      fhR[v] = fhatbar[(eR * NV + v) * Nf + fR];
    }
    pair_flux_vjp<D, T, NS, GEO>(uL, uR, n, mag, fhL, fhR, ph, uLb, uRb, fvL, fvR, nb, mb);
    if (GEO) {
      for (int j = 0; j < D; ++j) Gn[(eL * (D + 1) + j) * Nf + fL] += nb[j];
      Gn[(eL * (D + 1) + D) * Nf + fL] += mb / mag;
    }
    for (int v = 0; v < NV; ++v) {
      if (NS) {
        fvnbar[(eL * NV + v) * Nf + fL] = fvL[v];
        fvnbar[(eR * NV + v) * Nf + fR] = fvR[v];
      }
      ufbar[(eL * NV + v) * Nf + fL] = uLb[v];
      ufbar[(eR * NV + v) * Nf + fR] = uRb[v];
    }
  } else if (gid < npair + nbnd) {
    const int64_t b = gid - npair;
    const int32_t c = bnd[b];
    const int64_t e = c / Nf;
    const int fp = c % Nf;
    T uB[NV], n[D], fh[NV], uBb[NV], fv[NV], nb[D], mb = T(0);
    for (int j = 0; j < D; ++j) {
      n[j] = bnrm[b * (D + 1) + j];
      nb[j] = T(0);
    }
    const T mag = bnrm[b * (D + 1) + D];
    for (int v = 0; v < NV; ++v) {
      uB[v] = uf[(e * NV + v) * Nf + fp];
      fh[v] = fhatbar[(e * NV + v) * Nf + fp];
    }
    bnd_flux_vjp<D, T, NS, GEO>(uB, n, mag, fh, b < n_wall, flow[elem_mesh[e]], ph, uBb, fv, nb, mb);
    if (GEO) {
      for (int j = 0; j < D; ++j) Gn[(e * (D + 1) + j) * Nf + fp] += nb[j];
      Gn[(e * (D + 1) + D) * Nf + fp] += mb / mag;
    }
    for (int v = 0; v < NV; ++v) {
      ufbar[(e * NV + v) * Nf + fp] = uBb[v];
      if (NS) fvnbar[(e * NV + v) * Nf + fp] = fv[v];
    }
  }
}

template <int D, int P, typename T, int EE = 0>
struct VjpVolTile {
  using S = Shape<D, P>;
  // A: u + (u^ - u_f) | gradient | flux-point gradient adjoint | reference-gradient adjoint
  static constexpr int LA = cmax(cmax(S::NV * S::Ns + S::NV * S::Nf, D * S::NV * S::Ns), D * S::NV * S::Nf);
  // + own u_f + vol_bar + own u_f adjoint
  static constexpr int LE = LA + S::NV * S::Nf + S::NV * S::Ns + S::NV * S::Nf;
  static constexpr int E = EE > 0 ? EE : tile_elems<S::Ns>(LE, sizeof(T));
  static constexpr int BS = round64(cmax(E * S::Ns, E * S::Nf));
};

// Autotuner candidates of the NS volume adjoint (kind 3): (default tile, compiler's register
// budget), (half tile, compiler's budget), (default tile, a waves-per-SIMD launch bound one above
// the compiler's choice); degree 1 has the default only
template <int D, int P, typename T>
struct VCands {
  static constexpr int E0 = VjpVolTile<D, P, T>::E, E1 = E0 / 2 > 0 ? E0 / 2 : 1;
  static constexpr int W1 = sizeof(T) == 8 ? (D == 2 ? 3 : 2) : (D == 2 ? 5 : 3);
  static constexpr int N = P >= 3 ? 3 : 1;
  static void list(int32_t *out) {
    const int E[3] = {E0, E1, E0}, W[3] = {0, 0, W1};
    for (int c = 0; c < N; ++c) {
      out[3 * c] = E[c];
      out[3 * c + 1] = W[c];
      out[3 * c + 2] = 0;
    }
  }
  template <class F>
  static void pick(int c, F &&go) {
    if constexpr (N == 1) {
      go(std::integral_constant<int, E0>{}, std::integral_constant<int, 0>{});
    } else {
      if (c == 1)
        go(std::integral_constant<int, E1>{}, std::integral_constant<int, 0>{});
      else if (c == 2)
        go(std::integral_constant<int, E0>{}, std::integral_constant<int, W1>{});
      else
        go(std::integral_constant<int, E0>{}, std::integral_constant<int, 0>{});
    }
  }
};

// NS volume adjoint (see the file header), including the adjoint of the common flux at its own
// flux points: each point forms its pair's flux adjoint (both sides' u_f and common-flux adjoints,
// complete before this kernel) and keeps its own side's share, so no face kernel runs and each
// pair is differentiated once from each side.  Writes the solution-point adjoint ubvol (may alias
// volbar: each tile reads its vol_bar before writing), the own-flux-point adjoint ufb_own (must
// not alias fhatbar, which neighbouring tiles read) and the neighbour-slot adjoint ufb_nbr.
// GEO: also the metric adjoints (S rows from F~_k = S_k . F and from the gradient transform,
// 1/J from the gradient transform) into Gm, and the unit-normal and |N| adjoints of the common
// flux (at the L point of a pair and at boundary points), of the viscous normal flux and of the
// far-field states at own flux points into Gn
template <int D, int P, typename T, bool GEO, int EE>
__device__ __forceinline__ void vjp_ns_vol_body(
    const T *__restrict__ u, const T *__restrict__ uf, const int32_t *__restrict__ nbr, const T *__restrict__ fnrm,
    const T *__restrict__ bnrm, int64_t n_wall, const T *__restrict__ metric, const int32_t *__restrict__ elem_mesh,
    const FlowDev<T> *__restrict__ flow, const OpsDev<T, P> &ops_arg, const PhysDev<T> &ph, const T *volbar,
    const T *__restrict__ fhatbar, T *ubvol, T *__restrict__ ufb_own, T *__restrict__ ufb_nbr,
    T *__restrict__ Gm, T *__restrict__ Gn, int64_t Ne) {
  using S = Shape<D, P>;
  using TL = VjpVolTile<D, P, T, EE>;
  constexpr int E = TL::E, Ns = S::Ns, Nf = S::Nf, Nfp = S::Nfp, NV = S::NV, NM = S::NM;
  __shared__ __attribute__((aligned(16))) T lds[E * TL::LE];
  __shared__ OpsDev<T, P> ops;
  T *lA = lds;
  T *luf = lds + E * TL::LA;             // [E][NV][Nf]
  T *lvb = luf + E * NV * Nf;            // [E][NV][Ns]
  T *lub = lvb + E * NV * Ns;            // [E][NV][Nf] own u_f adjoint
  T *lu = lA;                            // [E][NV][Ns]
  T *ldu = lA + E * NV * Ns;             // [E][NV][Nf]
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (int)((Ne - e0) < E ? (Ne - e0) : E);
  __shared__ int s_mesh[E];  // mesh of each element (free-stream data)
  {
    // both tiles and the elements' mesh indices in one round trip
    TileLoad<E * NV * Ns, TL::BS, T> tu, tv;
    tu.load(u + e0 * NV * Ns, ne * NV * Ns);
    tv.load(volbar + e0 * NV * Ns, ne * NV * Ns);
    const int mesh = (int)threadIdx.x < ne ? elem_mesh[e0 + threadIdx.x] : 0;
    stage_ops(ops, ops_arg);
    tu.store(lu, ne * NV * Ns);
    tv.store(lvb, ne * NV * Ns);
    if ((int)threadIdx.x < ne) s_mesh[threadIdx.x] = mesh;
  }
  __syncthreads();
  const T wl = T(0.5) + ph.beta, wr = T(0.5) - ph.beta;
  // own u_f, LDG common solution, u^ - u_f (forward recompute)
  for (int idx = threadIdx.x; idx < ne * Nf; idx += blockDim.x) {
    const int el = idx / Nf, fp = idx % Nf;
    const int64_t e = e0 + el;
    int base, stride, side;
    line_of_fpt<D, P>(fp, base, stride, side);
    const T *lv = side ? ops.lp : ops.lm;
    T uo[NV], uh[NV];
    for (int v = 0; v < NV; ++v) {
      const T *lin = lu + (el * NV + v) * Ns + base;
      T s = T(0);
#pragma unroll
      for (int a = 0; a < P; ++a) s += lv[a] * lin[a * stride];
      uo[v] = s;
      luf[(el * NV + v) * Nf + fp] = s;
    }
    const int32_t code = nbr[e * Nf + fp];
    if (code >= 0) {
      const int32_t c = code & (NBR_R_BIT - 1);
      const int64_t e2 = c / Nf;
      const int f2 = c % Nf;
      const bool isR = (code & NBR_R_BIT) != 0;
      for (int v = 0; v < NV; ++v) {
        const T un = uf[(e2 * NV + v) * Nf + f2];
        uh[v] = isR ? wl * un + wr * uo[v] : wl * uo[v] + wr * un;
      }
    } else {
      const int64_t b = -(int64_t)code - 1;
      if (b < n_wall) {
        wall_state<D>(uo, uh);
      } else {
        T n[D];
        for (int j = 0; j < D; ++j) n[j] = bnrm[b * (D + 1) + j];
        farfield<D>(uo, n, flow[s_mesh[el]], ph.gamma, ph.gm1, uh);
      }
      for (int v = 0; v < NV; ++v) ufb_nbr[(e * NV + v) * Nf + fp] = T(0);  // no neighbour here
    }
    for (int v = 0; v < NV; ++v) ldu[(el * NV + v) * Nf + fp] = uh[v] - uo[v];
  }
  __syncthreads();
  const int el = threadIdx.x / Ns, i = threadIdx.x % Ns;
  const bool act = threadIdx.x < E * Ns && el < ne;
  const int64_t e = e0 + el;
  T uv[NV], gx[D][NV];
  if (act) {
    T Sm[D][D];
    for (int k = 0; k < D; ++k)
      for (int j = 0; j < D; ++j) Sm[k][j] = metric[(e * NM + k * D + j) * Ns + i];
    const T invJ = metric[(e * NM + D * D) * Ns + i];
    for (int j = 0; j < D; ++j)
      for (int v = 0; v < NV; ++v) gx[j][v] = T(0);
#pragma unroll 1
    for (int k = 0; k < D; ++k) {
      int base, stride, ik, t;
      line_of_sol<D, P>(i, k, base, stride, ik, t);
      const T cm = -ops.gm[ik], cp = ops.gp[ik];
      T Sk[D];
      pick_row<D>(Sm, k, Sk);
      for (int v = 0; v < NV; ++v) {
        const T *lin = lu + (el * NV + v) * Ns + base;
        T s = T(0);
#pragma unroll
        for (int a = 0; a < P; ++a) s += ops.D[ik * P + a] * lin[a * stride];
        const T *ld = ldu + (el * NV + v) * Nf;
        s += cm * ld[(2 * k) * Nfp + t] + cp * ld[(2 * k + 1) * Nfp + t];
        for (int j = 0; j < D; ++j) gx[j][v] += Sk[j] * s;
      }
    }
    for (int j = 0; j < D; ++j)
      for (int v = 0; v < NV; ++v) gx[j][v] *= invJ;
    for (int v = 0; v < NV; ++v) uv[v] = lu[(el * NV + v) * Ns + i];
  }
  __syncthreads();
  T *lg = lA;  // [E][D][NV][Ns] physical gradient
  if (act)
    for (int j = 0; j < D; ++j)
      for (int v = 0; v < NV; ++v) lg[((el * D + j) * NV + v) * Ns + i] = gx[j][v];
  __syncthreads();
  // adjoint of the viscous normal flux at own flux points (one flux point per thread)
  const int ef_idx = threadIdx.x;
  const bool actf = ef_idx < ne * Nf;
  T gbf[D * NV], stb[NV], nbv[D], ufa_face[NV];
  for (int j = 0; j < D; ++j) nbv[j] = T(0);
  int fpl = 0, elf = 0;
  if (actf) {
    elf = ef_idx / Nf;
    fpl = ef_idx % Nf;
    const int64_t ef = e0 + elf;
    int base, stride, side;
    line_of_fpt<D, P>(fpl, base, stride, side);
    const T *lv = side ? ops.lp : ops.lm;
    T g[D * NV], st[NV], n[D], fb[NV];
    for (int j = 0; j < D; ++j)
      for (int v = 0; v < NV; ++v) {
        const T *lin = lg + ((elf * D + j) * NV + v) * Ns + base;
        T s = T(0);
#pragma unroll
        for (int a = 0; a < P; ++a) s += lv[a] * lin[a * stride];
        g[j * NV + v] = s;
        gbf[j * NV + v] = T(0);
      }
    for (int v = 0; v < NV; ++v) {
      st[v] = luf[(elf * NV + v) * Nf + fpl];
      stb[v] = T(0);
    }
    for (int j = 0; j < D; ++j) n[j] = fnrm[(ef * (D + 1) + j) * Nf + fpl];
    const int32_t code = nbr[ef * Nf + fpl];
    {  // adjoint of this point's common flux: own u_f adjoint (face part) and fvn adjoint
      T fho[NV], nbc[D], mbc = T(0), dummy[NV];
      for (int v = 0; v < NV; ++v) fho[v] = fhatbar[(ef * NV + v) * Nf + fpl];
      for (int j = 0; j < D; ++j) nbc[j] = T(0);
      if (code >= 0) {
        const int32_t c = code & (NBR_R_BIT - 1);
        const int64_t e2 = c / Nf;
        const int f2 = c % Nf;
        const bool isR = (code & NBR_R_BIT) != 0;
        T un[NV], fhn[NV], nL[D];
        for (int v = 0; v < NV; ++v) {
          un[v] = uf[(e2 * NV + v) * Nf + f2];
          fhn[v] = fhatbar[(e2 * NV + v) * Nf + f2];
        }
        for (int j = 0; j < D; ++j) nL[j] = isR ? -n[j] : n[j];  // the pair's L normal (stored as -n_L on R)
        const T mag = fnrm[(ef * (D + 1) + D) * Nf + fpl];
        if (isR) {
          pair_flux_vjp<D, T, true, false>(un, st, nL, mag, fhn, fho, ph, dummy, ufa_face, dummy, fb, nbc, mbc);
        } else {
          pair_flux_vjp<D, T, true, GEO>(st, un, nL, mag, fho, fhn, ph, ufa_face, dummy, fb, dummy, nbc, mbc);
          if (GEO) {
            for (int j = 0; j < D; ++j) Gn[(ef * (D + 1) + j) * Nf + fpl] += nbc[j];
            Gn[(ef * (D + 1) + D) * Nf + fpl] += mbc / mag;
          }
        }
      } else {
        const int64_t b = -(int64_t)code - 1;
        T nB[D];
        for (int j = 0; j < D; ++j) nB[j] = bnrm[b * (D + 1) + j];
        const T mag = bnrm[b * (D + 1) + D];
        bnd_flux_vjp<D, T, true, GEO>(st, nB, mag, fho, b < n_wall, flow[s_mesh[elf]], ph, ufa_face, fb, nbc, mbc);
        if (GEO) {
          for (int j = 0; j < D; ++j) Gn[(ef * (D + 1) + j) * Nf + fpl] += nbc[j];
          Gn[(ef * (D + 1) + D) * Nf + fpl] += mbc / mag;
        }
      }
    }
    T ub[NV];
    bool heat = true, wall = false;
    int64_t b = -1;
    for (int v = 0; v < NV; ++v) ub[v] = st[v];
    if (code < 0) {
      b = -(int64_t)code - 1;
      if (b < n_wall) {
        wall_state<D>(st, ub);
        heat = false;
        wall = true;
      } else {
        farfield<D>(st, n, flow[s_mesh[elf]], ph.gamma, ph.gm1, ub);
      }
    }
    T ubb[NV];
    for (int v = 0; v < NV; ++v) ubb[v] = T(0);
    fvis_vjp<D>(ub, g, n, flow[s_mesh[elf]].mu, ph, heat, fb, ubb, gbf);
    if (GEO) {  // fvn = F_vis(ub, g) . n
      Visc<D, T> vs;
      visc_state<D>(ub, g, flow[s_mesh[elf]].mu, ph, heat, vs);
      fvis_columns_dot<D>(vs, fb, nbv);
      // the common flux is F^ . |N| and enters with this side's fvn_bar: |N|_bar += fvn_bar . fvn / |N|
      // (stored at this point; the node mapping folds an R point's share into its L partner)
      T fv[NV];
      fvis_dot<D>(vs, n, fv);
      T mb = T(0);
      for (int v = 0; v < NV; ++v) mb += fb[v] * fv[v];
      Gn[(ef * (D + 1) + D) * Nf + fpl] += mb / fnrm[(ef * (D + 1) + D) * Nf + fpl];
    }
    if (code < 0) {
      if (wall)
        wall_state_vjp<D>(st, ubb, stb);
      else
        farfield_vjp<D>(st, n, flow[s_mesh[elf]], ph.gamma, ph.gm1, ubb, stb, GEO ? nbv : nullptr);
    } else {
      for (int v = 0; v < NV; ++v) stb[v] = ubb[v];
    }
  }
  __syncthreads();
  T *lgb = lA;  // [E][D][NV][Nf] adjoint of the flux-point gradient
  if (actf) {
    for (int j = 0; j < D; ++j)
      for (int v = 0; v < NV; ++v) lgb[((elf * D + j) * NV + v) * Nf + fpl] = gbf[j * NV + v];
    for (int v = 0; v < NV; ++v) lub[(elf * NV + v) * Nf + fpl] = stb[v] + ufa_face[v];
  }
  __syncthreads();
  // solution points: F~_bar from vol_bar, pointwise flux adjoints, gradient adjoint
  T ubs[NV], grb[D][NV];
  if (act) {
    T Sm[D][D];
    for (int k = 0; k < D; ++k)
      for (int j = 0; j < D; ++j) Sm[k][j] = metric[(e * NM + k * D + j) * Ns + i];
    const T invJ = metric[(e * NM + D * D) * Ns + i];
    T gxb[D * NV];
    for (int q = 0; q < D * NV; ++q) gxb[q] = T(0);
    for (int v = 0; v < NV; ++v) ubs[v] = T(0);
    Visc<D, T> vs0;
    if (GEO) visc_state<D>(uv, &gx[0][0], flow[s_mesh[el]].mu, ph, true, vs0);
#pragma unroll 1
    for (int k = 0; k < D; ++k) {
      int base, stride, ik, t;
      line_of_sol<D, P>(i, k, base, stride, ik, t);
      T ftb[NV];
      for (int v = 0; v < NV; ++v) {
        const T *lin = lvb + (el * NV + v) * Ns + base;
        T sd = T(0);  // transpose of the divergence with the folded correction
#pragma unroll
        for (int a = 0; a < P; ++a) sd += ops.Dt[a * P + ik] * lin[a * stride];
        ftb[v] = sd;
      }
      if (GEO) {  // F~_k = S_k . (F_inv - F_vis):  S_k_bar += F^T F~_k_bar
        T sk[D], sv[D];
        for (int j = 0; j < D; ++j) sk[j] = sv[j] = T(0);
        finv_columns_dot<D>(uv, ph.gm1, ftb, sk);
        fvis_columns_dot<D>(vs0, ftb, sv);
        for (int j = 0; j < D; ++j) Gm[(e * NM + k * D + j) * Ns + i] += sk[j] - sv[j];
      }
      T Sk[D];
      pick_row<D>(Sm, k, Sk);
      finv_dot_vjp<D>(uv, Sk, ph.gm1, ftb, ubs);
      for (int v = 0; v < NV; ++v) ftb[v] = -ftb[v];
      fvis_vjp<D>(uv, &gx[0][0], Sk, flow[s_mesh[el]].mu, ph, true, ftb, ubs, gxb);
      // flux-point gradient adjoint back to this solution point (M0^T along the k-line)
      for (int j = 0; j < D; ++j)
        for (int v = 0; v < NV; ++v) {
          const T *lgf = lgb + ((el * D + j) * NV + v) * Nf;
          gxb[j * NV + v] += ops.lm[ik] * lgf[(2 * k) * Nfp + t] + ops.lp[ik] * lgf[(2 * k + 1) * Nfp + t];
        }
    }
    // grad_x u = J^-1 S^T grad_xi u  ->  reference-gradient adjoint
    for (int k = 0; k < D; ++k)
      for (int v = 0; v < NV; ++v) {
        T s = T(0);
        for (int j = 0; j < D; ++j) s += Sm[k][j] * gxb[j * NV + v];
        grb[k][v] = invJ * s;
      }
    if (GEO) {
      // S_bar[k][j] += (1/J) sum_v grad_xi_k u_v gxb[j][v] with grad_xi u = A^T grad_x u;
      // (1/J)_bar += sum gxb . grad_x u / (1/J)
      T A[D][D];
      jacobian_from_metric<D>(Sm, invJ, A);
      T gj = T(0);
      for (int j = 0; j < D; ++j)
        for (int v = 0; v < NV; ++v) gj += gxb[j * NV + v] * gx[j][v];
      Gm[(e * NM + D * D) * Ns + i] += gj / invJ;
      for (int k = 0; k < D; ++k) {
        T gk[NV];
        for (int v = 0; v < NV; ++v) {
          T s = T(0);
          for (int j = 0; j < D; ++j) s += A[j][k] * gx[j][v];
          gk[v] = s;
        }
        for (int j = 0; j < D; ++j) {
          T s = T(0);
          for (int v = 0; v < NV; ++v) s += gk[v] * gxb[j * NV + v];
          Gm[(e * NM + k * D + j) * Ns + i] += invJ * s;
        }
      }
    }
  }
  __syncthreads();
  T *lrb = lA;  // [E][D][NV][Ns] reference-gradient adjoint
  if (act)
    for (int k = 0; k < D; ++k)
      for (int v = 0; v < NV; ++v) lrb[((el * D + k) * NV + v) * Ns + i] = grb[k][v];
  __syncthreads();
  if (act) {
    // D_k^T of the reference gradient
#pragma unroll 1
    for (int k = 0; k < D; ++k) {
      int base, stride, ik, t;
      line_of_sol<D, P>(i, k, base, stride, ik, t);
      for (int v = 0; v < NV; ++v) {
        const T *lin = lrb + ((el * D + k) * NV + v) * Ns + base;
        T s = T(0);
#pragma unroll
        for (int a = 0; a < P; ++a) s += ops.D[a * P + ik] * lin[a * stride];
        ubs[v] += s;
      }
    }
    for (int v = 0; v < NV; ++v) ubvol[(e * NV + v) * Ns + i] = ubs[v];
  }
  // lifting of (u^ - u_f): adjoint at flux points -> own and neighbour u_f adjoints
  if (actf) {
    const int64_t ef = e0 + elf;
    int base, stride, side;
    line_of_fpt<D, P>(fpl, base, stride, side);
    const int k = (fpl / Nfp) >> 1;
    T dub[NV];
    for (int v = 0; v < NV; ++v) {
      const T *lin = lrb + ((elf * D + k) * NV + v) * Ns + base;
      T s = T(0);
#pragma unroll
      for (int a = 0; a < P; ++a) s += (side ? ops.gp[a] : -ops.gm[a]) * lin[a * stride];
      dub[v] = s;
    }
    T own[NV];
    for (int v = 0; v < NV; ++v) own[v] = lub[(elf * NV + v) * Nf + fpl] - dub[v];
    const int32_t code = nbr[ef * Nf + fpl];
    if (code >= 0) {
      const int32_t c = code & (NBR_R_BIT - 1);
      const int64_t e2 = c / Nf;
      const int f2 = c % Nf;
      const bool isR = (code & NBR_R_BIT) != 0;
      const T wo = isR ? wr : wl, wn = isR ? wl : wr;
      for (int v = 0; v < NV; ++v) {
        own[v] += wo * dub[v];
        ufb_nbr[(e2 * NV + v) * Nf + f2] = wn * dub[v];
      }
    } else {
      const int64_t b = -(int64_t)code - 1;
      T st[NV];
      for (int v = 0; v < NV; ++v) st[v] = luf[(elf * NV + v) * Nf + fpl];
      if (b < n_wall) {
        wall_state_vjp<D>(st, dub, own);
      } else {
        T n[D];
        for (int j = 0; j < D; ++j) n[j] = bnrm[b * (D + 1) + j];
        farfield_vjp<D>(st, n, flow[s_mesh[elf]], ph.gamma, ph.gm1, dub, own, GEO ? nbv : nullptr);
      }
    }
    for (int v = 0; v < NV; ++v) ufb_own[(ef * NV + v) * Nf + fpl] = own[v];
    if (GEO)
      for (int j = 0; j < D; ++j) Gn[(ef * (D + 1) + j) * Nf + fpl] += nbv[j];
  }
}

// the NS volume adjoint with the compiler's register budget, and with a waves-per-SIMD launch
// bound WW (an autotuner candidate); same body
template <int D, int P, typename T, bool GEO, int EE = 0>
__global__ __launch_bounds__((VjpVolTile<D, P, T, EE>::BS)) void k_vjp_ns_vol(
    const T *__restrict__ u, const T *__restrict__ uf, const int32_t *__restrict__ nbr, const T *__restrict__ fnrm,
    const T *__restrict__ bnrm, int64_t n_wall, const T *__restrict__ metric, const int32_t *__restrict__ elem_mesh,
    const FlowDev<T> *__restrict__ flow, OpsDev<T, P> ops_arg, PhysDev<T> ph, const T *volbar,
    const T *__restrict__ fhatbar, T *ubvol, T *__restrict__ ufb_own, T *__restrict__ ufb_nbr,
    T *__restrict__ Gm, T *__restrict__ Gn, int64_t Ne) {
  vjp_ns_vol_body<D, P, T, GEO, EE>(u, uf, nbr, fnrm, bnrm, n_wall, metric, elem_mesh, flow, ops_arg, ph, volbar,
                                    fhatbar, ubvol, ufb_own, ufb_nbr, Gm, Gn, Ne);
}
template <int D, int P, typename T, bool GEO, int EE, int WW>
__global__ __launch_bounds__((VjpVolTile<D, P, T, EE>::BS), WW) void k_vjp_ns_vol_w(
    const T *__restrict__ u, const T *__restrict__ uf, const int32_t *__restrict__ nbr, const T *__restrict__ fnrm,
    const T *__restrict__ bnrm, int64_t n_wall, const T *__restrict__ metric, const int32_t *__restrict__ elem_mesh,
    const FlowDev<T> *__restrict__ flow, OpsDev<T, P> ops_arg, PhysDev<T> ph, const T *volbar,
    const T *__restrict__ fhatbar, T *ubvol, T *__restrict__ ufb_own, T *__restrict__ ufb_nbr,
    T *__restrict__ Gm, T *__restrict__ Gn, int64_t Ne) {
  vjp_ns_vol_body<D, P, T, GEO, EE>(u, uf, nbr, fnrm, bnrm, n_wall, metric, elem_mesh, flow, ops_arg, ph, volbar,
                                    fhatbar, ubvol, ufb_own, ufb_nbr, Gm, Gn, Ne);
}

// launches the NS volume adjoint with the solver's chosen candidate
template <int D, int P, typename T, bool GEO>
void launch_vjp_ns_vol(const fr_solver *s, hipStream_t st, const T *u, const T *uf, const T *metric,
                       const FlowDev<T> *fl, const OpsDev<T, P> &o, const PhysDev<T> &ph, const T *volbar,
                       const T *fhatbar, T *ubvol, T *ufb_own, T *ufb_nbr, T *Gm, T *Gn) {
  VCands<D, P, T>::pick(s->tune[3], [&](auto te, auto tw) {
    constexpr int EE = decltype(te)::value, WW = decltype(tw)::value;
    using TV = VjpVolTile<D, P, T, EE>;
    const unsigned nb = (unsigned)((s->Ne + TV::E - 1) / TV::E);
    if constexpr (WW == 0)
      k_vjp_ns_vol<D, P, T, GEO, EE><<<nb, TV::BS, 0, st>>>(
          u, uf, s->nbr, (const T *)s->fnrm, (const T *)s->bnd_nrm, s->n_wall, metric, s->elem_mesh, fl, o, ph,
          volbar, fhatbar, ubvol, ufb_own, ufb_nbr, Gm, Gn, s->Ne);
    else
      k_vjp_ns_vol_w<D, P, T, GEO, EE, WW><<<nb, TV::BS, 0, st>>>(
          u, uf, s->nbr, (const T *)s->fnrm, (const T *)s->bnd_nrm, s->n_wall, metric, s->elem_mesh, fl, o, ph,
          volbar, fhatbar, ubvol, ufb_own, ufb_nbr, Gm, Gn, s->Ne);
  });
}
// Euler volume adjoint: F~_bar from vol_bar, pointwise inviscid-flux adjoint
template <int D, int P, typename T, bool GEO>
__global__ __launch_bounds__((VjpDivTile<D, P, T>::BS)) void k_vjp_euler_vol(const T *__restrict__ u,
                                                                             const T *__restrict__ metric,
                                                                             OpsDev<T, P> ops_arg, PhysDev<T> ph,
                                                                             const T *volbar, T *ubvol,
                                                                             T *__restrict__ Gm, int64_t Ne) {
  using S = Shape<D, P>;
  using TL = VjpDivTile<D, P, T>;
  constexpr int E = TL::E, Ns = S::Ns, NV = S::NV, NM = S::NM;
  __shared__ __attribute__((aligned(16))) T lvb[E * TL::LE];
  __shared__ OpsDev<T, P> ops;
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (int)((Ne - e0) < E ? (Ne - e0) : E);
  const int el = threadIdx.x / Ns, i = threadIdx.x % Ns;
  const int64_t e = e0 + el;
  // the adjoint tile and this point's state in one round trip
  TileLoad<E * NV * Ns, TL::BS, T> tv;
  tv.load(volbar + e0 * NV * Ns, ne * NV * Ns);
  T uv[NV], ubs[NV];
  for (int v = 0; v < NV; ++v) {
    uv[v] = el < ne ? u[(e * NV + v) * Ns + i] : T(0);
    ubs[v] = T(0);
  }
  stage_ops(ops, ops_arg);
  tv.store(lvb, ne * NV * Ns);
  __syncthreads();
  if (el >= ne) return;
  for (int k = 0; k < D; ++k) {
    T Sk[D];
    for (int j = 0; j < D; ++j) Sk[j] = metric[(e * NM + k * D + j) * Ns + i];
    int base, stride, ik, t;
    line_of_sol<D, P>(i, k, base, stride, ik, t);
    T ftb[NV];
    for (int v = 0; v < NV; ++v) {
      const T *lin = lvb + (el * NV + v) * Ns + base;
      T sd = T(0);  // transpose of the divergence with the folded correction
#pragma unroll
      for (int a = 0; a < P; ++a) sd += ops.Dt[a * P + ik] * lin[a * stride];
      ftb[v] = sd;
    }
    if (GEO) {  // S_k_bar += F_inv^T F~_k_bar
      T sk[D];
      for (int j = 0; j < D; ++j) sk[j] = T(0);
      finv_columns_dot<D>(uv, ph.gm1, ftb, sk);
      for (int j = 0; j < D; ++j) Gm[(e * NM + k * D + j) * Ns + i] += sk[j];
    }
    finv_dot_vjp<D>(uv, Sk, ph.gm1, ftb, ubs);
  }
  for (int v = 0; v < NV; ++v) ubvol[(e * NV + v) * Ns + i] = ubs[v];
}

// RK4-step adjoint epilogue of the VJP: with z = (dR/du)^T k_bar of this stage,
// u_bar += z and the previous stage's k_bar = dt (ca a + cz z) (a = dJ/du_{n+1})
template <typename T>
struct AdjRK {
  T *a, *kb, *ub;
  const double *dt;  // per mesh
  const int32_t *elem_mesh;
  T ca, cz;
};

// z = ubvol + M0^T (ufb_own + ufb_nbr); u_bar += z, or the RK epilogue when rk.ub is set
template <int D, int P, typename T>
__global__ __launch_bounds__((VjpDivTile<D, P, T>::BS)) void k_vjp_final(const T *ubvol, const T *__restrict__ ufb_own,
                                                                         const T *__restrict__ ufb_nbr,
                                                                         OpsDev<T, P> ops_arg, T *__restrict__ ubar,
                                                                         AdjRK<T> rk, int64_t Ne) {
  using S = Shape<D, P>;
  using TL = VjpDivTile<D, P, T>;
  constexpr int E = TL::E, Ns = S::Ns, Nf = S::Nf, Nfp = S::Nfp, NV = S::NV;
  __shared__ OpsDev<T, P> ops;
  stage_ops(ops, ops_arg);
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (int)((Ne - e0) < E ? (Ne - e0) : E);
  const int el = threadIdx.x / Ns, i = threadIdx.x % Ns;
  if (el >= ne) return;
  const int64_t e = e0 + el;
  // every operand of the point is requested before the first product
  int ik[D], fm[D], fpp[D];
  for (int k = 0; k < D; ++k) {
    int base, stride, t;
    line_of_sol<D, P>(i, k, base, stride, ik[k], t);
    fm[k] = (2 * k) * Nfp + t;
    fpp[k] = (2 * k + 1) * Nfp + t;
  }
  T sv[NV], am[NV][D], ap[NV][D], prev[NV];
  const int mesh = rk.ub ? rk.elem_mesh[e] : 0;
  for (int v = 0; v < NV; ++v) {
    const int64_t o = (e * NV + v) * Ns + i;
    sv[v] = ubvol[o];
    const T *fo = ufb_own + (e * NV + v) * Nf;
    for (int k = 0; k < D; ++k) {
      am[v][k] = fo[fm[k]];
      ap[v][k] = fo[fpp[k]];
    }
    if (ufb_nbr) {
      const T *fn = ufb_nbr + (e * NV + v) * Nf;
      for (int k = 0; k < D; ++k) {
        am[v][k] += fn[fm[k]];
        ap[v][k] += fn[fpp[k]];
      }
    }
    prev[v] = rk.ub ? rk.a[o] : ubar[o];
  }
  const T dt = rk.ub ? (T)rk.dt[mesh] : T(0);
  for (int v = 0; v < NV; ++v) {
    T s = sv[v];
    for (int k = 0; k < D; ++k) s += ops.lm[ik[k]] * am[v][k] + ops.lp[ik[k]] * ap[v][k];
    const int64_t o = (e * NV + v) * Ns + i;
    if (rk.ub) {
      rk.ub[o] += s;
      if (rk.kb) rk.kb[o] = dt * (rk.ca * prev[v] + rk.cz * s);
    } else {
      ubar[o] = prev[v] + s;
    }
  }
}

// Epilogue of reverse stage k of an RK4 step fused with the first reverse kernel of stage k-1 on
// the same element tile: z = ubvol + M0^T (ufb_own + ufb_nbr), u_bar += z, and the next stage's
// r_bar = dt (ca a + cz z) is consumed at once: w = -(1/J) r_bar -> vol_bar, F^_bar = Lift^T w at
// the flux points, and the flux-point values u_f = M0 y of the next linearisation state y.
// vol_bar aliases ubvol: each tile reads its own elements' values before the barrier that precedes
// its writes.  GEO: the adjoint of 1/J of stage k-1 (r_bar . R / (1/J)).
template <int D, int P, typename T, bool GEO>
__global__ __launch_bounds__((VjpDivTile<D, P, T>::BS)) void k_vjp_final_div(
    const T *ubvol, const T *ufb_own, const T *__restrict__ ufb_nbr, OpsDev<T, P> ops_arg, AdjRK<T> rk,
    const T *__restrict__ y, const T *__restrict__ metric, T *volbar, T *fhatbar, T *__restrict__ uf,
    const T *__restrict__ Rf, T *__restrict__ Gm, int64_t Ne) {
  using S = Shape<D, P>;
  using TL = VjpDivTile<D, P, T>;
  constexpr int E = TL::E, Ns = S::Ns, Nf = S::Nf, Nfp = S::Nfp, NV = S::NV, NM = S::NM;
  __shared__ __attribute__((aligned(16))) T lw[E * TL::LE];
  __shared__ __attribute__((aligned(16))) T lu[E * TL::LE];
  __shared__ OpsDev<T, P> ops;
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (int)((Ne - e0) < E ? (Ne - e0) : E);
  const int el = threadIdx.x / Ns, i = threadIdx.x % Ns;
  const int64_t e = e0 + el;
  // the next state's tile and every operand of this point in one round trip
  TileLoad<E * NV * Ns, TL::BS, T> tu;
  tu.load(y + e0 * NV * Ns, ne * NV * Ns);
  int ik[D], fm[D], fpp[D];
  T sv[NV], am[NV][D], ap[NV][D], prev[NV], rf[NV];
  T invJ = T(0), gprev = T(0), dt = T(0);
  if (el < ne) {
    for (int k = 0; k < D; ++k) {
      int base, stride, t;
      line_of_sol<D, P>(i, k, base, stride, ik[k], t);
      fm[k] = (2 * k) * Nfp + t;
      fpp[k] = (2 * k + 1) * Nfp + t;
    }
    dt = (T)rk.dt[rk.elem_mesh[e]];
    invJ = metric[(e * NM + D * D) * Ns + i];
    for (int v = 0; v < NV; ++v) {
      const int64_t o = (e * NV + v) * Ns + i;
      sv[v] = ubvol[o];
      const T *fo = ufb_own + (e * NV + v) * Nf;
      for (int k = 0; k < D; ++k) {
        am[v][k] = fo[fm[k]];
        ap[v][k] = fo[fpp[k]];
      }
      if (ufb_nbr) {
        const T *fn = ufb_nbr + (e * NV + v) * Nf;
        for (int k = 0; k < D; ++k) {
          am[v][k] += fn[fm[k]];
          ap[v][k] += fn[fpp[k]];
        }
      }
      prev[v] = rk.a[o];
      if (GEO) rf[v] = Rf[o];
    }
    if (GEO) gprev = Gm[(e * NM + D * D) * Ns + i];
  }
  stage_ops(ops, ops_arg);
  tu.store(lu, ne * NV * Ns);
  __syncthreads();
  if (el < ne) {
    T gj = T(0);
    for (int v = 0; v < NV; ++v) {
      T z = sv[v];
      for (int k = 0; k < D; ++k) z += ops.lm[ik[k]] * am[v][k] + ops.lp[ik[k]] * ap[v][k];
      const int64_t o = (e * NV + v) * Ns + i;
      rk.ub[o] += z;
      const T rb = dt * (rk.ca * prev[v] + rk.cz * z);
      const T w = -invJ * rb;
      lw[(el * NV + v) * Ns + i] = w;
      volbar[o] = w;
      if (GEO) gj += rb * rf[v];
    }
    if (GEO) Gm[(e * NM + D * D) * Ns + i] = gprev + gj / invJ;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < ne * NV * Nf; idx += blockDim.x) {
    const int fp = idx % Nf, rest = idx / Nf;
    int base, stride, side;
    line_of_fpt<D, P>(fp, base, stride, side);
    const T *g = side ? ops.gp : ops.gm;
    const T *lv = side ? ops.lp : ops.lm;
    const T *lin = lw + rest * Ns + base;
    const T *lun = lu + rest * Ns + base;
    T sw = T(0), su = T(0);
#pragma unroll
    for (int a = 0; a < P; ++a) {
      sw += g[a] * lin[a * stride];
      su += lv[a] * lun[a * stride];
    }
    fhatbar[e0 * NV * Nf + idx] = sw;
    uf[e0 * NV * Nf + idx] = su;
  }
}

// ------------------------------------------------------------------------------------ launcher
static inline unsigned vblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <int D, int P, typename T>
struct VjpEngine {
  using S = Shape<D, P>;
  static void run(const fr_solver *s, const T *u, const T *rbar, T *ubar, T *work, const AdjRK<T> &rk,
                  const GeoVjpArgs &geo, hipStream_t st) {
    if (geo.Gm)
      run_t<true>(s, u, rbar, ubar, work, rk, geo, st);
    else
      run_t<false>(s, u, rbar, ubar, work, rk, geo, st);
  }

  template <bool GEO>
  static void run_t(const fr_solver *s, const T *u, const T *rbar, T *ubar, T *work, const AdjRK<T> &rk,
                    const GeoVjpArgs &geo, hipStream_t st) {
    const OpsDev<T, P> o = make_ops<T, P>(s->ops);
    PhysDev<T> ph;
    ph.gamma = (T)s->gamma;
    ph.gm1 = (T)(s->gamma - 1.0);
    ph.prandtl = (T)s->prandtl;
    ph.beta = (T)s->beta;
    ph.tau = (T)s->tau;
    ph.side = ldg_side_of<T>(s->beta);
    const int64_t Ne = s->Ne, nsol = Ne * S::NV * S::Ns, nf = Ne * S::NV * S::Nf;
    T *volbar = work;            // also the solution-point adjoint (read before write per tile)
    T *fhatbar = volbar + nsol;  // also the own flux-point adjoint
    T *ufbface = fhatbar + nf;
    T *fvnbar = ufbface + nf;
    T *ufbnbr = fvnbar + nf;
    // forward flux-point state of the linearisation point, [Ne][NV][Nf], filled by k_vjp_div.
    // The reverse sweep touches only its own work arrays, so a forward recording of another
    // state may run concurrently on another stream (the trajectory adjoint overlaps the
    // recompute of one checkpoint segment with the reverse sweep of the next).
    T *uf = ufbnbr + nf;
    const T *metric = (const T *)s->metric;
    const FlowDev<T> *fl = (const FlowDev<T> *)s->flow;
    T *Gm = (T *)geo.Gm, *Gn = (T *)geo.Gn;
    const T *Rf = (const T *)geo.R;
    using TD = VjpDivTile<D, P, T>;
    k_vjp_div<D, P, T, GEO><<<vblk(Ne, TD::E), TD::BS, 0, st>>>(rbar, u, metric, o, volbar, fhatbar, uf, Rf, Gm, Ne);
    const int64_t nface = s->npair + s->nbnd;
    if (s->equations == 1) {
      launch_vjp_ns_vol<D, P, T, GEO>(s, st, u, uf, metric, fl, o, ph, volbar, fhatbar, volbar, ufbface, ufbnbr,
                                      Gm, Gn);
      k_vjp_final<D, P, T><<<vblk(Ne, TD::E), TD::BS, 0, st>>>(volbar, ufbface, ufbnbr, o, ubar, rk, Ne);
    } else {
      k_vjp_face<D, P, T, false, GEO><<<vblk(nface, 256), 256, 0, st>>>(
          uf, fhatbar, s->pairL, s->pairR, (const T *)s->pair_nrm, s->npair, s->bnd, (const T *)s->bnd_nrm,
          s->n_wall, s->nbnd, s->elem_mesh, fl, ph, ufbface, nullptr, Gn);
      k_vjp_euler_vol<D, P, T, GEO><<<vblk(Ne, TD::E), TD::BS, 0, st>>>(u, metric, o, ph, volbar, volbar, Gm, Ne);
      k_vjp_final<D, P, T><<<vblk(Ne, TD::E), TD::BS, 0, st>>>(volbar, ufbface, nullptr, o, ubar, rk, Ne);
    }
  }
};

// The reverse sweep of one RK4 step (stages 4..1): the first stage's div kernel forms its r_bar
// from the entry adjoint (no separate combine kernel), and every later stage's div work is fused
// into the epilogue of the stage before it; with the face adjoint inside the Navier-Stokes volume
// adjoint a step is 1 + 4 x 2 = 9 launches (Euler: 1 + 4 x 3).
template <int D, int P, typename T>
struct VjpStepEngine {
  using S = Shape<D, P>;
  template <bool GEO>
  static void run(const fr_solver *s, const T *const ys[4], T *ub, T *A, const double *dt, const T *const Rs[4],
                  T *Gm, T *Gn, T *work, hipStream_t st) {
    const OpsDev<T, P> o = make_ops<T, P>(s->ops);
    PhysDev<T> ph;
    ph.gamma = (T)s->gamma;
    ph.gm1 = (T)(s->gamma - 1.0);
    ph.prandtl = (T)s->prandtl;
    ph.beta = (T)s->beta;
    ph.tau = (T)s->tau;
    ph.side = ldg_side_of<T>(s->beta);
    const int64_t Ne = s->Ne, nsol = Ne * S::NV * S::Ns, nf = Ne * S::NV * S::Nf;
    T *volbar = work, *fhatbar = volbar + nsol, *ufbface = fhatbar + nf, *fvnbar = ufbface + nf;
    T *ufbnbr = fvnbar + nf, *uf = ufbnbr + nf;
    const T *metric = (const T *)s->metric;
    const FlowDev<T> *fl = (const FlowDev<T> *)s->flow;
    static const double cA[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    static const double cZ[4] = {0.5, 0.5, 1.0, 0.0};
    using TD = VjpDivTile<D, P, T>;
    const bool ns = s->equations == 1;
    k_vjp_div<D, P, T, GEO, true><<<vblk(Ne, TD::E), TD::BS, 0, st>>>(
        ub, ys[3], metric, o, volbar, fhatbar, uf, GEO ? Rs[3] : nullptr, Gm, Ne, A, dt, s->elem_mesh, (T)cA[3]);
    const int64_t nface = s->npair + s->nbnd;
    for (int k = 3; k >= 0; --k) {
      T *own = ufbface;  // own flux-point adjoint (NS volume adjoint, or the Euler face adjoint)
      T *nbr = ns ? ufbnbr : nullptr;
      if (ns) {
        launch_vjp_ns_vol<D, P, T, GEO>(s, st, ys[k], uf, metric, fl, o, ph, volbar, fhatbar, volbar, ufbface,
                                        ufbnbr, Gm, Gn);
      } else {
        k_vjp_face<D, P, T, false, GEO><<<vblk(nface, 256), 256, 0, st>>>(
            uf, fhatbar, s->pairL, s->pairR, (const T *)s->pair_nrm, s->npair, s->bnd, (const T *)s->bnd_nrm,
            s->n_wall, s->nbnd, s->elem_mesh, fl, ph, ufbface, nullptr, Gn);
        k_vjp_euler_vol<D, P, T, GEO><<<vblk(Ne, TD::E), TD::BS, 0, st>>>(ys[k], metric, o, ph, volbar, volbar,
                                                                          Gm, Ne);
      }
      if (k > 0) {
        AdjRK<T> rk{A, nullptr, ub, dt, s->elem_mesh, (T)cA[k - 1], (T)cZ[k - 1]};
        k_vjp_final_div<D, P, T, GEO><<<vblk(Ne, TD::E), TD::BS, 0, st>>>(
            volbar, own, nbr, o, rk, ys[k - 1], metric, volbar, fhatbar, uf, GEO ? Rs[k - 1] : nullptr, Gm, Ne);
      } else {
        AdjRK<T> rk{A, nullptr, ub, dt, s->elem_mesh, T(0), T(0)};
        k_vjp_final<D, P, T><<<vblk(Ne, TD::E), TD::BS, 0, st>>>(volbar, own, nbr, o, nullptr, rk, Ne);
      }
    }
  }
};

// work-array size in elements of the state type
size_t vjp_work_elems(const fr_solver *s) {
  return (size_t)s->Ne * s->NV * (s->Ns + 5 * s->Nf);
}

// u_bar += (dR/du (u))^T r_bar when rk_a is NULL.  Otherwise the RK4-step adjoint epilogue:
// with z = (dR/du (u))^T r_bar, rk_ub += z and rk_kb = dt (ca rk_a + cz z) (rk_kb may be r_bar:
// it is read by the first kernel and written by the last).
bool launch_vjp(const fr_solver *s, const void *u, const void *rbar, void *ubar, void *work, const void *rk_a,
                void *rk_kb, void *rk_ub, double ca, double cz, const double *dt, const GeoVjpArgs &geo,
                hipStream_t st) {
#define FR_VCASE(DD, PP)                                                                              \
  if (s->dim == DD && s->p + 1 == PP) {                                                               \
    if (s->precision == 0) {                                                                          \
      AdjRK<double> rk{(double *)rk_a, (double *)rk_kb, (double *)(rk_a ? rk_ub : nullptr), dt,       \
                       s->elem_mesh, ca, cz};                                                         \
      VjpEngine<DD, PP, double>::run(s, (const double *)u, (const double *)rbar, (double *)ubar,      \
                                     (double *)work, rk, geo, st);                                    \
    } else {                                                                                          \
      AdjRK<float> rk{(float *)rk_a, (float *)rk_kb, (float *)(rk_a ? rk_ub : nullptr), dt,           \
                      s->elem_mesh, (float)ca, (float)cz};                                            \
      VjpEngine<DD, PP, float>::run(s, (const float *)u, (const float *)rbar, (float *)ubar,          \
                                    (float *)work, rk, geo, st);                                      \
    }                                                                                                 \
    return true;                                                                                      \
  }
  FR_VCASE(2, 2) FR_VCASE(2, 3) FR_VCASE(2, 4) FR_VCASE(2, 5)
  FR_VCASE(3, 2) FR_VCASE(3, 3) FR_VCASE(3, 4) FR_VCASE(3, 5)
#undef FR_VCASE
  return false;
}

// u_bar <- (d u_{n+1} / d u_n)^T u_bar for one RK4 step with stage states ys[0..3] (ys[0] = u_n);
// A: state-sized scratch for the entry adjoint.  With Gm / Gn (mesh-node adjoint) the stage
// residuals Rs[0..3] are required.
bool launch_vjp_rk_step(const fr_solver *s, const void *const ys[4], void *u_bar, void *A, const double *dt,
                        const void *const Rs[4], void *Gm, void *Gn, void *work, hipStream_t st) {
#define FR_SCASE(DD, PP)                                                                                  \
  if (s->dim == DD && s->p + 1 == PP) {                                                                   \
    if (s->precision == 0) {                                                                              \
      using T = double;                                                                                   \
      const T *y[4] = {(const T *)ys[0], (const T *)ys[1], (const T *)ys[2], (const T *)ys[3]};           \
      const T *r[4] = {nullptr, nullptr, nullptr, nullptr};                                               \
      if (Rs) for (int k = 0; k < 4; ++k) r[k] = (const T *)Rs[k];                                         \
      if (Gm) VjpStepEngine<DD, PP, T>::run<true>(s, y, (T *)u_bar, (T *)A, dt, r, (T *)Gm, (T *)Gn, (T *)work, st); \
      else VjpStepEngine<DD, PP, T>::run<false>(s, y, (T *)u_bar, (T *)A, dt, r, nullptr, nullptr, (T *)work, st); \
    } else {                                                                                              \
      using T = float;                                                                                    \
      const T *y[4] = {(const T *)ys[0], (const T *)ys[1], (const T *)ys[2], (const T *)ys[3]};           \
      const T *r[4] = {nullptr, nullptr, nullptr, nullptr};                                               \
      if (Rs) for (int k = 0; k < 4; ++k) r[k] = (const T *)Rs[k];                                         \
      if (Gm) VjpStepEngine<DD, PP, T>::run<true>(s, y, (T *)u_bar, (T *)A, dt, r, (T *)Gm, (T *)Gn, (T *)work, st); \
      else VjpStepEngine<DD, PP, T>::run<false>(s, y, (T *)u_bar, (T *)A, dt, r, nullptr, nullptr, (T *)work, st); \
    }                                                                                                     \
    return true;                                                                                          \
  }
  FR_SCASE(2, 2) FR_SCASE(2, 3) FR_SCASE(2, 4) FR_SCASE(2, 5)
  FR_SCASE(3, 2) FR_SCASE(3, 3) FR_SCASE(3, 4) FR_SCASE(3, 5)
#undef FR_SCASE
  return false;
}

int vjp_tune_cands(const fr_solver *s, int32_t *cand) {
#define FR_TCASE(DD, PP)                                            \
  if (s->dim == DD && s->p + 1 == PP) {                             \
    if (s->precision == 0) {                                        \
      VCands<DD, PP, double>::list(cand);                           \
      return VCands<DD, PP, double>::N;                             \
    }                                                               \
    VCands<DD, PP, float>::list(cand);                              \
    return VCands<DD, PP, float>::N;                                \
  }
  FR_TCASE(2, 2) FR_TCASE(2, 3) FR_TCASE(2, 4) FR_TCASE(2, 5)
  FR_TCASE(3, 2) FR_TCASE(3, 3) FR_TCASE(3, 4) FR_TCASE(3, 5)
#undef FR_TCASE
  return 0;
}

}  // namespace frmi
