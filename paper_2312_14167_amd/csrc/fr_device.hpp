// Device-side building blocks shared by the forward and adjoint kernels: element shapes, line
// indexing of the tensor-product operators, pointwise Navier-Stokes physics, LDS staging.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fr_solver.hpp"

namespace frmi {


template <int D_, int P_>
struct Shape {
  static constexpr int D = D_, P = P_;
  static constexpr int Ns = (D == 2) ? P * P : P * P * P;
  static constexpr int Nfp = (D == 2) ? P : P * P;
  static constexpr int Nf = 2 * D * Nfp;
  static constexpr int NV = D + 2;
  static constexpr int NM = D * D + 1;
};

// index of value (e, v, fp) in the flux-point layout of u_f and the common flux (see
// uf_face_skip): face-blocked where faces fill two lines, else [Ne][NV][Nf]
template <int D, int P, typename T>
struct UfLayout {
  using S = Shape<D, P>;
  static constexpr int NFACE = 2 * D, FB = S::NV * S::Nfp;
  static constexpr bool SKIP = uf_face_skip(FB, (int)sizeof(T));  // face-blocked, faces skipped
  static constexpr int FS = uf_face_stride(FB, (int)sizeof(T));   // face stride (face-blocked)
  static constexpr int EB = NFACE * FS;                            // element stride
  static constexpr int VS = SKIP ? S::Nfp : S::Nf;                 // variable stride
  static constexpr int FST = SKIP ? FS : S::Nfp;                   // face stride of one variable
  // offset of point fp of element e (variable 0); variable v adds v * VS
  __device__ __forceinline__ static int64_t point(int64_t e, int fp) {
    if constexpr (SKIP) return e * EB + (fp / S::Nfp) * FST + fp % S::Nfp;
    else return e * EB + fp;
  }
  __device__ __forceinline__ static int64_t at(int64_t e, int v, int fp) { return point(e, fp) + v * VS; }
};

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int round64(int x) { return (x + 63) / 64 * 64; }

// elements per workgroup for an LDS footprint of `vals` values of `bytes` each
template <int Ns>
constexpr int tile_elems(int vals, int bytes) {
  return cmax(1, cmin(512 / Ns, (60 * 1024) / (vals * bytes)));
}

// line through solution point i along reference coordinate k: first point and stride
template <int D, int P>
__device__ __forceinline__ void line_of_sol(int i, int k, int &base, int &stride, int &ik, int &t) {
  const int i0 = i % P, i1 = (i / P) % P, i2 = i / (P * P);
  if (k == 0) { stride = 1; ik = i0; t = (D == 2) ? i1 : i1 + P * i2; }
  else if (k == 1) { stride = P; ik = i1; t = (D == 2) ? i0 : i0 + P * i2; }
  else { stride = P * P; ik = i2; t = i0 + P * i1; }
  base = i - ik * stride;
}

// line of flux point fp (face f = fp / Nfp): first solution point, stride, side (0: -1, 1: +1)
template <int D, int P>
__device__ __forceinline__ void line_of_fpt(int fp, int &base, int &stride, int &side) {
  constexpr int Nfp = (D == 2) ? P : P * P;
  const int f = fp / Nfp, t = fp % Nfp, k = f >> 1;
  side = f & 1;
  if (D == 2) {
    if (k == 0) { base = P * t; stride = 1; }
    else { base = t; stride = P; }
  } else {
    if (k == 0) { base = P * t; stride = 1; }
    else if (k == 1) { base = (t % P) + P * P * (t / P); stride = P; }
    else { base = t; stride = P * P; }
  }
}

// ------------------------------------------------------------------------------------ physics
template <int D, typename T>
__device__ __forceinline__ void primitives(const T *u, T gm1, T &rho, T *v, T &p) {
  rho = u[0];
  const T ir = T(1) / rho;
  T ke = T(0);
  for (int j = 0; j < D; ++j) { v[j] = u[1 + j] * ir; ke += v[j] * u[1 + j]; }
  p = gm1 * (u[D + 1] - T(0.5) * ke);
}

// inviscid flux (Eq. (3)) dotted with a vector m (unit normal, or a metric row S_k)
template <int D, typename T>
__device__ __forceinline__ void finv_dot(const T *u, const T *m, T gm1, T *out) {
  T rho, v[D], p;
  primitives<D>(u, gm1, rho, v, p);
  T vm = T(0);
  for (int j = 0; j < D; ++j) vm += v[j] * m[j];
  out[0] = u[0] * vm;
  for (int i = 0; i < D; ++i) out[1 + i] = u[1 + i] * vm + p * m[i];
  out[D + 1] = (u[D + 1] + p) * vm;
}

// viscous quantities at a point from the state u and conserved gradient g[j*NV + v]
template <int D, typename T>
struct Visc {
  T v[D];
  T tau[D][D];
  T q[D];
};

template <int D, typename T>
__device__ __forceinline__ void visc_state(const T *u, const T *g, T mu, const PhysDev<T> &ph, bool heat,
                                           Visc<D, T> &o) {
  constexpr int NV = D + 2;
  const T ir = T(1) / u[0];
  const T Es = u[D + 1] * ir;
  T dv[D][D], dth[D];
  for (int i = 0; i < D; ++i) o.v[i] = u[1 + i] * ir;
  for (int j = 0; j < D; ++j) {
    const T gr = g[j * NV + 0];
    T s = T(0);
    for (int i = 0; i < D; ++i) {
      dv[i][j] = (g[j * NV + 1 + i] - o.v[i] * gr) * ir;
      s += o.v[i] * dv[i][j];
    }
    const T de = (g[j * NV + D + 1] - Es * gr) * ir;
    dth[j] = ph.gm1 * (de - s);
  }
  T div = T(0);
  for (int i = 0; i < D; ++i) div += dv[i][i];
  const T c23 = T(2) / T(3);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j)
      o.tau[i][j] = mu * (dv[i][j] + dv[j][i] - (i == j ? c23 * div : T(0)));
  const T kappa = heat ? mu * ph.gamma / (ph.prandtl * ph.gm1) : T(0);
  for (int j = 0; j < D; ++j) o.q[j] = -kappa * dth[j];
}

// viscous flux (0, tau_ij, u_i tau_ij - q_j) dotted with m
template <int D, typename T>
__device__ __forceinline__ void fvis_dot(const Visc<D, T> &o, const T *m, T *out) {
  out[0] = T(0);
  T en = T(0);
  for (int i = 0; i < D; ++i) {
    T s = T(0);
    for (int j = 0; j < D; ++j) s += o.tau[i][j] * m[j];
    out[1 + i] = s;
    en += o.v[i] * s;
  }
  for (int j = 0; j < D; ++j) en -= o.q[j] * m[j];
  out[D + 1] = en;
}

// viscous normal flux F_vis(st, grad) . n with the flux-point gradient produced one derivative
// direction at a time (grad_d(v) = gdir(d, v)); keeps 8 accumulators instead of the full
// gradient and stress tensor:
//   (tau n)_i = mu (sum_j d_j v_i n_j + sum_j d_i v_j n_j - 2/3 div n_i),
//   energy    = v . (tau n) + kappa d_n(p/rho)   (zero heat flux when !heat)
template <int D, typename T, class G>
__device__ __forceinline__ void fvis_normal_stream(const T *st, const G &gdir, const T *n, T mu,
                                                   const PhysDev<T> &ph, bool heat, T *fv) {
  constexpr int NV = D + 2;
  const T ir = T(1) / st[0];
  const T Es = st[D + 1] * ir;
  T vel[D], dvn[D], dvT[D];
  for (int m = 0; m < D; ++m) { vel[m] = st[1 + m] * ir; dvn[m] = T(0); }
  T div = T(0), dthn = T(0);
#pragma unroll 1
  for (int d = 0; d < D; ++d) {
    T gd[NV];
    gdir(d, gd);
    T sv = T(0), tn = T(0);
    for (int m = 0; m < D; ++m) {
      const T dvdm = (gd[1 + m] - vel[m] * gd[0]) * ir;  // d_d v_m
      sv += vel[m] * dvdm;
      dvn[m] += dvdm * n[d];
      tn += dvdm * n[m];
      if (m == d) div += dvdm;
    }
    dvT[d] = tn;
    const T dth = ph.gm1 * ((gd[D + 1] - Es * gd[0]) * ir - sv);
    dthn += dth * n[d];
  }
  const T c23 = T(2) / T(3);
  T en = T(0);
  fv[0] = T(0);
  for (int i = 0; i < D; ++i) {
    const T t = mu * (dvn[i] + dvT[i] - c23 * div * n[i]);
    fv[1 + i] = t;
    en += vel[i] * t;
  }
  const T kappa = heat ? mu * ph.gamma / (ph.prandtl * ph.gm1) : T(0);
  fv[D + 1] = en + kappa * dthn;
}

template <int D, typename T>
__device__ __forceinline__ void rusanov(const T *uL, const T *uR, const T *n, T gamma, T gm1, T *F) {
  // primitives once per side; the sound speed reuses the reciprocal density
  const T irL = T(1) / uL[0], irR = T(1) / uR[0];
  T vnL = T(0), vnR = T(0), keL = T(0), keR = T(0);
  for (int j = 0; j < D; ++j) {
    const T vl = uL[1 + j] * irL, vr = uR[1 + j] * irR;
    keL += vl * uL[1 + j];
    keR += vr * uR[1 + j];
    vnL += vl * n[j];
    vnR += vr * n[j];
  }
  const T pL = gm1 * (uL[D + 1] - T(0.5) * keL), pR = gm1 * (uR[D + 1] - T(0.5) * keR);
  const T aL = fabs(vnL) + sqrt(gamma * pL * irL);
  const T aR = fabs(vnR) + sqrt(gamma * pR * irR);
  const T lam = aL >= aR ? aL : aR;
  F[0] = T(0.5) * (uL[0] * vnL + uR[0] * vnR) - T(0.5) * lam * (uR[0] - uL[0]);
  for (int i = 0; i < D; ++i)
    F[1 + i] = T(0.5) * ((uL[1 + i] * vnL + pL * n[i]) + (uR[1 + i] * vnR + pR * n[i])) -
               T(0.5) * lam * (uR[1 + i] - uL[1 + i]);
  F[D + 1] = T(0.5) * ((uL[D + 1] + pL) * vnL + (uR[D + 1] + pR) * vnR) - T(0.5) * lam * (uR[D + 1] - uL[D + 1]);
}

// Riemann-invariant far-field state
template <int D, typename T>
__device__ __forceinline__ void farfield(const T *uL, const T *n, const FlowDev<T> &fl, T gamma, T gm1, T *ub) {
  T rL, vL[D], pL;
  primitives<D>(uL, gm1, rL, vL, pL);
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
  const T rho = pow(c * c / (gamma * s), T(1) / gm1);
  const T p = rho * c * c / gamma;
  T ke = T(0);
  ub[0] = rho;
  for (int j = 0; j < D; ++j) {
    const T vt = out ? vL[j] - vnL * n[j] : fl.v[j] - vni * n[j];
    const T vj = vt + vn * n[j];
    ub[1 + j] = rho * vj;
    ke += vj * vj;
  }
  ub[D + 1] = p / gm1 + T(0.5) * rho * ke;
}

// operator tables staged in LDS: per-lane dynamic indexing into them is an LDS read instead of
// a register-resident copy of every coefficient
template <typename T, int P>
__device__ __forceinline__ void stage_ops(OpsDev<T, P> &dst, const OpsDev<T, P> &src) {
  constexpr int n = (int)(sizeof(OpsDev<T, P>) / sizeof(T));
  const T *s = reinterpret_cast<const T *>(&src);
  T *d = reinterpret_cast<T *>(&dst);
  for (int k = threadIdx.x; k < n; k += blockDim.x) d[k] = s[k];
}

// contiguous tile copy global -> LDS of n <= NMAX elements by a BS-thread block, split in two so
// that a kernel requests all of its start-up loads before the first wait: load() issues every
// element load of this thread, store() puts them into LDS (one memory round trip per tile instead
// of one per loop iteration)
template <int NMAX, int BS, typename T>
struct TileLoad {
  static constexpr int K = (NMAX + BS - 1) / BS;
  T r[K];
  __device__ __forceinline__ void load(const T *__restrict__ src, int n) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int idx = (int)threadIdx.x + k * BS;
      if (idx < n) r[k] = src[(uint32_t)idx];
    }
  }
  __device__ __forceinline__ void store(T *__restrict__ dst, int n) const {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int idx = (int)threadIdx.x + k * BS;
      if (idx < n) dst[idx] = r[k];
    }
  }
};

// no-slip wall state: zero velocity, same density and internal energy
template <int D, typename T>
__device__ __forceinline__ void wall_state(const T *uB, T *uw) {
  T ke = T(0);
  for (int j = 0; j < D; ++j) ke += uB[1 + j] * uB[1 + j];
  uw[0] = uB[0];
  for (int j = 0; j < D; ++j) uw[1 + j] = T(0);
  uw[D + 1] = uB[D + 1] - T(0.5) * ke / uB[0];
}

}  // namespace frmi
