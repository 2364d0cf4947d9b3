// Mesh-node adjoint: from the adjoints of the metric terms at solution points (S rows and 1/J)
// and of the unit normal and |N| at flux points to the adjoint of every node coordinate.
//
// Forward chain (Eq. (1) in transformed form, degree-q Lagrange map on GLL nodes):
//   A[j][k] = dx_j/dxi_k = sum_n X_{n,j} dphi_n/dxi_k;  S = adj(A);  1/J = 1/det(A)
//   flux point of face f (coordinate k_f, side s_f):  N = s_f S_f[k_f, :],  |N|,  n = N / |N|
// Interior face pairs use the L side's normal and |N| on both sides, so the R side's adjoints
// are folded into the L point's (its normal is -n_L).  Per element, one workgroup forms A_bar at
// every solution and owning flux point, then dphi^T A_bar at every element node; a second kernel
// sums each node's contributions over its elements in a fixed order (no atomics).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fr_device.hpp"
#include "fr_dispatch.hpp"

namespace frmi {

// S = adj(A): row k of S; returns det A
template <int D>
__device__ __forceinline__ double adj_fwd(const double (&A)[D][D], double (&S)[D][D]) {
  if (D == 2) {
    S[0][0] = A[1][1];
    S[0][1] = -A[0][1];
    S[1][0] = -A[1][0];
    S[1][1] = A[0][0];
    return A[0][0] * A[1][1] - A[0][1] * A[1][0];
  } else {
    // row k = column k+1 x column k+2 (cyclic)
    for (int k = 0; k < D; ++k) {
      const int a = (k + 1) % D, b = (k + 2) % D;
      S[k][0] = A[1][a] * A[2][b] - A[2][a] * A[1][b];
      S[k][1] = A[2][a] * A[0][b] - A[0][a] * A[2][b];
      S[k][2] = A[0][a] * A[1][b] - A[1][a] * A[0][b];
    }
    return S[0][0] * A[0][0] + S[0][1] * A[1][0] + S[0][2] * A[2][0];
  }
}

// Ab += d(sum_kj Sb[k][j] adj(A)[k][j]) / dA
template <int D>
__device__ __forceinline__ void adj_vjp(const double (&A)[D][D], const double (&Sb)[D][D], double (&Ab)[D][D]) {
  if (D == 2) {
    Ab[1][1] += Sb[0][0];
    Ab[0][1] -= Sb[0][1];
    Ab[1][0] -= Sb[1][0];
    Ab[0][0] += Sb[1][1];
  } else {
    // c = u x v with u = column a, v = column b:  u_bar += v x c_bar,  v_bar += c_bar x u
    for (int k = 0; k < D; ++k) {
      const int a = (k + 1) % D, b = (k + 2) % D;
      const double *cb = Sb[k];
      Ab[0][a] += A[1][b] * cb[2] - A[2][b] * cb[1];
      Ab[1][a] += A[2][b] * cb[0] - A[0][b] * cb[2];
      Ab[2][a] += A[0][b] * cb[1] - A[1][b] * cb[0];
      Ab[0][b] += cb[1] * A[2][a] - cb[2] * A[1][a];
      Ab[1][b] += cb[2] * A[0][a] - cb[0] * A[2][a];
      Ab[2][b] += cb[0] * A[1][a] - cb[1] * A[0][a];
    }
  }
}

constexpr int GEO_MAX_NN = 125;  // (q+1)^dim for q <= 4 in 3-D

template <int D, int P, typename T>
__global__ __launch_bounds__(256) void k_geo_nodes(const T *__restrict__ Gm, const T *__restrict__ Gn,
                                                   const int32_t *__restrict__ nbr, const double *__restrict__ Xe,
                                                   const double *__restrict__ dphi_s, const double *__restrict__ dphi_f,
                                                   int nn, double *__restrict__ Xeb) {
  using S = Shape<D, P>;
  constexpr int Ns = S::Ns, Nf = S::Nf, Nfp = S::Nfp, NM = S::NM;
  __shared__ double sAb[(Ns + Nf) * D * D];
  __shared__ double sX[GEO_MAX_NN * D];
  const int64_t e = blockIdx.x;
  for (int idx = threadIdx.x; idx < nn * D; idx += blockDim.x) sX[idx] = Xe[e * nn * D + idx];
  __syncthreads();
  for (int a = threadIdx.x; a < Ns + Nf; a += blockDim.x) {
    const bool sol = a < Ns;
    const int pt = sol ? a : a - Ns;
    const double *dp = sol ? dphi_s : dphi_f;
    const int npts = sol ? Ns : Nf;
    double A[D][D], Ab[D][D];
    for (int j = 0; j < D; ++j)
      for (int k = 0; k < D; ++k) {
        double s = 0.0;
        for (int n = 0; n < nn; ++n) s += dp[((int64_t)k * npts + pt) * nn + n] * sX[n * D + j];
        A[j][k] = s;
        Ab[j][k] = 0.0;
      }
    double Sm[D][D];
    const double J = adj_fwd<D>(A, Sm);
    if (sol) {
      double Sb[D][D];
      for (int k = 0; k < D; ++k)
        for (int j = 0; j < D; ++j) Sb[k][j] = (double)Gm[(e * NM + k * D + j) * Ns + pt];
      adj_vjp<D>(A, Sb, Ab);
      // 1/J = 1/det A:  d(1/J)/dA[j][k] = -(1/J)^2 adj(A)[k][j]
      const double ib = (double)Gm[(e * NM + D * D) * Ns + pt];
      const double c = -ib / (J * J);
      for (int j = 0; j < D; ++j)
        for (int k = 0; k < D; ++k) Ab[j][k] += c * Sm[k][j];
    } else {
      const int32_t code = nbr[e * Nf + pt];
      const bool owns = code < 0 || (code & NBR_R_BIT) == 0;
      if (owns) {
        const int f = pt / Nfp, kf = f >> 1;
        const double sf = (f & 1) ? 1.0 : -1.0;
        double N[D], nrm = 0.0;
        for (int j = 0; j < D; ++j) {
          N[j] = sf * Sm[kf][j];
          nrm += N[j] * N[j];
        }
        const double mag = sqrt(nrm);
        double nb[D], dot = 0.0;
        for (int j = 0; j < D; ++j) nb[j] = (double)Gn[(e * (D + 1) + j) * Nf + pt];
        double mb = (double)Gn[(e * (D + 1) + D) * Nf + pt];
        if (code >= 0) {  // the R partner used -n_L and |N_L|
          const int32_t c2 = code & (NBR_R_BIT - 1);
          const int64_t e2 = c2 / Nf;
          const int f2 = c2 % Nf;
          for (int j = 0; j < D; ++j) nb[j] -= (double)Gn[(e2 * (D + 1) + j) * Nf + f2];
          mb += (double)Gn[(e2 * (D + 1) + D) * Nf + f2];
        }
        for (int j = 0; j < D; ++j) dot += nb[j] * N[j] / mag;
        double Sb[D][D];
        for (int k = 0; k < D; ++k)
          for (int j = 0; j < D; ++j) Sb[k][j] = 0.0;
        for (int j = 0; j < D; ++j) {
          const double nj = N[j] / mag;
          Sb[kf][j] = sf * ((nb[j] - dot * nj) / mag + mb * nj);
        }
        adj_vjp<D>(A, Sb, Ab);
      }
    }
    for (int j = 0; j < D; ++j)
      for (int k = 0; k < D; ++k) sAb[(a * D + j) * D + k] = Ab[j][k];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nn * D; idx += blockDim.x) {
    const int n = idx / D, j = idx % D;
    double s = 0.0;
    for (int a = 0; a < Ns + Nf; ++a) {
      const bool sol = a < Ns;
      const int pt = sol ? a : a - Ns;
      const double *dp = sol ? dphi_s : dphi_f;
      const int npts = sol ? Ns : Nf;
      for (int k = 0; k < D; ++k) s += dp[((int64_t)k * npts + pt) * nn + n] * sAb[(a * D + j) * D + k];
    }
    Xeb[(e * nn + n) * D + j] = s;
  }
}

// x_bar[node] += sum of the node's per-element contributions, in incidence order
__global__ void k_geo_gather(const double *__restrict__ Xeb, const int32_t *__restrict__ inc_ptr,
                             const int32_t *__restrict__ inc, int64_t n_node, int dim, double *__restrict__ xbar) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= n_node) return;
  for (int j = 0; j < dim; ++j) {
    double s = 0.0;
    for (int32_t t = inc_ptr[node]; t < inc_ptr[node + 1]; ++t) s += Xeb[(int64_t)inc[t] * dim + j];
    xbar[node * dim + j] += s;
  }
}

template <int D, int P, typename T>
static void run_geo_nodes(const fr_solver *s, double *x_bar, hipStream_t st) {
  k_geo_nodes<D, P, T><<<(unsigned)s->Ne, 256, 0, st>>>((const T *)s->geo_Gm, (const T *)s->geo_Gn, s->nbr, s->geo_Xe,
                                                        s->geo_dphi_s, s->geo_dphi_f, s->geo_nn, s->geo_Xeb);
  k_geo_gather<<<(unsigned)((s->n_node + 255) / 256), 256, 0, st>>>(s->geo_Xeb, s->geo_inc_ptr, s->geo_inc,
                                                                     s->n_node, s->dim, x_bar);
}

bool launch_geo_nodes(const fr_solver *s, double *x_bar, hipStream_t st) {
  if (s->geo_nn > GEO_MAX_NN) return false;
#define FR_GCASE(DD, PP)                                                        \
  if (s->dim == DD && s->p + 1 == PP) {                                         \
    if (s->precision == 0) run_geo_nodes<DD, PP, double>(s, x_bar, st);         \
    else run_geo_nodes<DD, PP, float>(s, x_bar, st);                            \
    return true;                                                                \
  }
  FR_GCASE(2, 2) FR_GCASE(2, 3) FR_GCASE(2, 4) FR_GCASE(2, 5)
  FR_GCASE(3, 2) FR_GCASE(3, 3) FR_GCASE(3, 4) FR_GCASE(3, 5)
#undef FR_GCASE
  return false;
}

}  // namespace frmi
