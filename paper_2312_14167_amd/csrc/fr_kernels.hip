// HIP kernels for CDNA4 (gfx950): FR residual stages, RK4 update, probe and force accumulators.
//
// Data layout (element-major, per-element blocks are contiguous so a workgroup's tile of
// elements is one contiguous range of HBM):
//   state, residual, RK arrays, volume term   [Ne][NV][Ns]
//   u_f, common flux, viscous normal flux     UfLayout: [Ne][2 dim][face block], each face block
//                                             [NV][Nfp] padded to whole 128-byte lines, where a
//                                             face fills two lines; else [Ne][NV][Nf]
//   metrics                                   [Ne][dim*dim + 1][Ns] (S = adj(dx/dxi) row-major, 1/J)
//   neighbour codes [Ne][Nf] (int32), outward unit normals and |N| [Ne][dim + 1][Nf]
// Element operators are applied in sum-factorised (tensor-product) form along the P points of
// each reference line: every operator is a P x P contraction per line, so the whole stage is
// bound by HBM traffic and on-chip latency, not by arithmetic.  Volume kernels stage their
// element tile in LDS once and read all line operands from LDS.
//
// Stage pipeline (Navier-Stokes), one launch each:
//   interp      u_f = M0 u (only before the first stage of a call; later stages get u_f from
//               div_rk)
//   ns_grad     per element tile: own u_f = M0 u; LDG common solution u^ from the neighbour's u_f
//               or the boundary state; corrected gradient grad_xi u = D_k u + s_f g_R'(s_f xi)
//               (u^ - u_f); grad_x u = J^-1 S^T grad_xi u; viscous normal flux at the flux points
//               whose value the common flux uses; with the one-sided LDG flux (beta = +-1/2) the
//               flux side also forms its pair's whole common flux (Rusanov - LDG viscous +
//               penalty) x |N|; F~_k = S_k . (F_inv - F_vis); vol = sum_k D~_k F~_k (the
//               correction's interior part folded into D~)
//   face_flux   two-sided LDG (beta != +-1/2): common normal flux per pair and boundary point
//   div_rk      R = -(1/J) (vol + Lift F^_n); RK4 stage update; u_f of the new stage state
// Euler: face_flux, then euler_vol_rk (F~, vol, lifting and the RK update in one kernel).

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fr_device.hpp"
#include "fr_dispatch.hpp"

namespace frmi {

// ------------------------------------------------------------------------------------ kernels
// common normal flux x |N| at every flux point.  Inviscid: Rusanov with the neighbour state or
// the boundary ghost.  NS: minus the LDG viscous flux assembled from the per-side viscous normal
// fluxes fvn (each side's F_vis(u, grad u) . n_out, boundary points already in boundary form).
template <int D, int P, typename T, bool NS>
__global__ __launch_bounds__(256, 6) void k_face_flux(const T *__restrict__ uf, const T *__restrict__ fvn,
                                                   const int32_t *__restrict__ pairL, const int32_t *__restrict__ pairR,
                                                   const T *__restrict__ pnrm, int64_t npair,
                                                   const int32_t *__restrict__ bnd, const T *__restrict__ bnrm,
                                                   int64_t n_wall, int64_t nbnd, const int32_t *__restrict__ elem_mesh,
                                                   const FlowDev<T> *__restrict__ flow, PhysDev<T> ph,
                                                   T *__restrict__ fhat) {
  using S = Shape<D, P>;
  constexpr int NV = S::NV, Nf = S::Nf;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < npair) {
    const int32_t cL = pairL[gid], cR = pairR[gid];
    const int64_t eL = cL / Nf, eR = cR / Nf;
    const int fL = cL % Nf, fR = cR % Nf;
    T uL[NV], uR[NV], n[D], F[NV];
    for (int v = 0; v < NV; ++v) {
      uL[v] = uf[UfLayout<D, P, T>::at(eL, v, fL)];
      uR[v] = uf[UfLayout<D, P, T>::at(eR, v, fR)];
    }
    for (int j = 0; j < D; ++j) n[j] = pnrm[gid * (D + 1) + j];
    const T mag = pnrm[gid * (D + 1) + D];
    rusanov<D>(uL, uR, n, ph.gamma, ph.gm1, F);
    if (NS) {
      // F^_vis . n_L = (1/2 - b) fvn_L + (1/2 + b) (-fvn_R) - tau (u_L - u_R)
      const T wl = T(0.5) - ph.beta, wr = T(0.5) + ph.beta;
      // a side with zero weight (one-sided LDG) never had its fvn computed: not read
      if (wl == T(0)) {
        for (int v = 0; v < NV; ++v) F[v] -= -wr * fvn[UfLayout<D, P, T>::at(eR, v, fR)] - ph.tau * (uL[v] - uR[v]);
      } else if (wr == T(0)) {
        for (int v = 0; v < NV; ++v) F[v] -= wl * fvn[UfLayout<D, P, T>::at(eL, v, fL)] - ph.tau * (uL[v] - uR[v]);
      } else {
        for (int v = 0; v < NV; ++v) {
          const T fl = fvn[UfLayout<D, P, T>::at(eL, v, fL)];
          const T fr = fvn[UfLayout<D, P, T>::at(eR, v, fR)];
          F[v] -= wl * fl - wr * fr - ph.tau * (uL[v] - uR[v]);
        }
      }
    }
    for (int v = 0; v < NV; ++v) {
      fhat[UfLayout<D, P, T>::at(eL, v, fL)] = F[v] * mag;
      fhat[UfLayout<D, P, T>::at(eR, v, fR)] = -F[v] * mag;
    }
  } else if (gid < npair + nbnd) {
    const int64_t b = gid - npair;
    const int32_t c = bnd[b];
    const int64_t e = c / Nf;
    const int fp = c % Nf;
    T uB[NV], ug[NV], n[D], F[NV];
    for (int v = 0; v < NV; ++v) uB[v] = uf[UfLayout<D, P, T>::at(e, v, fp)];
    for (int j = 0; j < D; ++j) n[j] = bnrm[b * (D + 1) + j];
    const T mag = bnrm[b * (D + 1) + D];
    if (b < n_wall) {
      ug[0] = uB[0];
      for (int j = 0; j < D; ++j) ug[1 + j] = -uB[1 + j];
      ug[D + 1] = uB[D + 1];
    } else {
      farfield<D>(uB, n, flow[elem_mesh[e]], ph.gamma, ph.gm1, ug);
    }
    rusanov<D>(uB, ug, n, ph.gamma, ph.gm1, F);
    if (NS)
      for (int v = 0; v < NV; ++v) F[v] -= fvn[UfLayout<D, P, T>::at(e, v, fp)];
    for (int v = 0; v < NV; ++v) fhat[UfLayout<D, P, T>::at(e, v, fp)] = F[v] * mag;
  }
}

// tile sizes (elements per workgroup E) of the LDS-staged volume kernels: EE = 0 gives the
// default; the autotuner also tries the default's halves and quarters (TileCands)
template <int D, int P, typename T, int EE = 0, int WW = 0>
struct GradTile {
  using S = Shape<D, P>;
  // per element: the state [NV][Ns], kept to the flux-point viscous phase, then one region that
  // holds u^ - u_f [NV][Nf] (with the tile's neighbour codes [Nf] behind all elements' u^ - u_f),
  // the physical gradient point-major [Ns][D][NV] and the transformed flux [D][NV][Ns] in turn;
  // in 2-D also the metric terms S [D*D][Ns], which each thread keeps there from the gradient to
  // the transformed flux, and the first phase's partial common flux [NV][Nf] for the viscous
  // flux-point phase (2-D tiles are small enough that this costs no occupancy; 3-D re-reads S
  // and passes the partial flux through fhat).  The default E fits four workgroups in 160 KB.
  static constexpr bool KEEP2D = D == 2;
  static constexpr int LU = S::NV * S::Ns;
  static constexpr int LC = (S::Nf * (int)sizeof(int32_t) + (int)sizeof(T) - 1) / (int)sizeof(T);
  static constexpr int LG = cmax(S::NV * S::Nf + LC, D * S::NV * S::Ns);
  static constexpr int LS = KEEP2D ? D * D * S::Ns + S::NV * S::Nf : 0;
  static constexpr int LE = LU + LG + LS;
  // degree 0 (a degree group of a variable-degree mesh): at most 16 elements, so that a group of
  // ten thousand elements still spreads over every CU
  static constexpr int E0 = cmax(1, cmin(512 / S::Ns, (40 * 1024 - 640) / (LE * (int)sizeof(T))));
  static constexpr int E = EE > 0 ? EE : (P == 1 ? cmin(E0, 16) : E0);
  static constexpr int BS = round64(E * S::Ns);
  // register budget (launch bound, waves per SIMD): 4 (128 VGPRs) in FP64, 7 (72 VGPRs) in FP32
  // by default; WW > 0 (an autotuner candidate) sets it
  static constexpr int MIN_WAVES = WW > 0 ? WW : (sizeof(T) == 4 ? 7 : 4);
};

// index of a thread's flux point in pass `pass` over a face-list-ordered tile: odd passes walk the
// threads backwards, so that the points beyond one pass land on the last wave, which holds the
// cheap end of the list (faces without gather or flux work), and not on wave 0, which holds the
// costly front.  Pass k covers [k BS, (k+1) BS), so a thread's index grows with the pass.
template <int BS>
__device__ __forceinline__ int flux_pass_index(int pass) {
  const int t = (int)threadIdx.x;
  return pass * BS + ((pass & 1) ? BS - 1 - t : t);
}

template <int D, int P, typename T, int EE = 0>
struct DivTile {
  using S = Shape<D, P>;
  static constexpr int LE = cmax(UfLayout<D, P, T>::EB, S::NV * S::Ns);  // common-flux tile, then state
  // degree 0: at most 32 elements per workgroup (see GradTile)
  static constexpr int E = EE > 0 ? EE : (P == 1 ? cmin(tile_elems<S::Ns>(LE, sizeof(T)), 32)
                                                  : tile_elems<S::Ns>(LE, sizeof(T)));
  static constexpr int BS = round64(E * S::Ns);
};

template <int D, int P, typename T, int EE = 0>
struct EulerTile {
  using S = Shape<D, P>;
  static constexpr int LE = D * S::NV * S::Ns + UfLayout<D, P, T>::EB;
  static constexpr int E = EE > 0 ? EE : tile_elems<S::Ns>(LE, sizeof(T));
  static constexpr int BS = round64(E * S::Ns);
};

// autotuner candidates: the default E, its half and its quarter
template <int E0>
struct TileCands {
  static constexpr int c0 = E0, c1 = cmax(1, E0 / 2), c2 = cmax(1, E0 / 4);
};

// Volume divergence vol = sum_k Dt_k F~_k on the matrix cores (FP32, 3-D): for each element and
// direction k, the line operator Dt (P x P, zero-padded to 16 rows x 8) times the tile's line
// values (columns = (variable, line), 16 per tile) in v_mfma_f32_16x16x4f32 steps (two K steps of
// 4 line points).  One wave per (element, column tile); the directions are summed in LDS (acc,
// [E][NV][Ns]) in the order 0, 1, 2 with a barrier between them, so the result is deterministic.
// lw holds F~ as [E][D][NV][Ns].  Lane layout of the 16x16x4 FP32 step: A[r][q] from lane r + 16 q,
// B[q][c] from lane c + 16 q, D[r][c] in lane c + 16 (r / 4), component r % 4.
template <int D, int P, int BS>
__device__ __forceinline__ void mfma_divergence(const float *lw, float *acc, const float *Dt, int ne, int E) {
  static_assert(D == 3 && P <= 8, "matrix-core divergence: 3-D, at most 8 points per line");
  using S = Shape<D, P>;
  constexpr int NV = S::NV, Ns = S::Ns, NL = Ns / P, NCOL = NV * NL, NT = (NCOL + 15) / 16, NW = BS / 64;
  typedef float f4 __attribute__((ext_vector_type(4)));
  const int wave = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
  const int r = lane % 16, q = lane / 16, c = lane % 16;
  // this lane's A entries of the two K steps (rows beyond P and points beyond P are zero)
  const float a0 = (r < P && q < P) ? Dt[r * P + q] : 0.f;
  const float a1 = (r < P && q + 4 < P) ? Dt[r * P + q + 4] : 0.f;
  for (int k = 0; k < D; ++k) {
    const int stride = k == 0 ? 1 : (k == 1 ? P : P * P);
    for (int item = wave; item < E * NT; item += NW) {
      const int el = item / NT, tile = item % NT;
      if (el >= ne) break;  // items are element-major: the rest of this wave's items are empty too
      const int col = tile * 16 + c;
      const bool cv = col < NCOL;
      const int v = cv ? col / NL : 0, line = cv ? col % NL : 0;
      const int base = k == 0 ? P * line : (k == 1 ? (line % P) + P * P * (line / P) : line);
      const float *src = lw + ((el * D + k) * NV + v) * Ns + base;
      const float b0 = (cv && q < P) ? src[q * stride] : 0.f;
      const float b1 = (cv && q + 4 < P) ? src[(q + 4) * stride] : 0.f;
      f4 d = {0.f, 0.f, 0.f, 0.f};
      d = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, d, 0, 0, 0);
      if (cv) {
        float *dst = acc + (el * NV + v) * Ns + base;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = 4 * q + j;
          if (row < P) dst[row * stride] = (k == 0) ? d[j] : dst[row * stride] + d[j];
        }
      }
    }
    __syncthreads();
  }
}

// NS volume kernel.  Per element tile:
//   own u_f = M0 u; LDG common solution from the neighbour's u_f (or the boundary state);
//   corrected gradient grad_xi u = D_k u + s_f g_R'(s_f xi)(u^ - u_f); grad_x u = J^-1 S^T grad_xi u;
//   viscous normal flux fvn = F_vis(u_f, M0 grad_x u) . n_out at the own flux points whose value
//   the common viscous flux uses (walls: zero-velocity state, no heat flux; far field: Riemann
//   state); F~_k = S_k . (F_inv - F_vis) at solution points;
//   vol = sum_k D~_k F~_k with D~ = D - (interior part of the correction), i.e.
//   vol = sum_k D_k F~_k - Lift (s_f M0 F~_{k_f}).
// MORTAR (a degree group of a mesh with several solution degrees): boundary points from n_bc on
// lie on faces to another degree; their common solution comes from ifc_uh ([point][NV], written by
// the mortar kernels), their viscous normal flux is stored like a boundary point's, and their
// common flux is left to the mortar kernels.
// WW: waves-per-SIMD launch bound (0: the precision's default); MFMA_DIV: the volume divergence on
// the matrix cores (FP32, 3-D; an autotuner candidate)
template <int D, int P, typename T, int EE, bool MORTAR = false, int WW = 0, bool MFMA_DIV = false>
__global__ __launch_bounds__((GradTile<D, P, T, EE>::BS), (GradTile<D, P, T, EE, WW>::MIN_WAVES)) void k_ns_grad(
    const T *__restrict__ u, const T *__restrict__ uf, const int32_t *__restrict__ nbr, const T *__restrict__ fnrm,
    const T *__restrict__ bnrm, int64_t n_wall, const T *__restrict__ metric, const int32_t *__restrict__ elem_mesh,
    const FlowDev<T> *__restrict__ flow, OpsDev<T, P> ops_arg, PhysDev<T> ph, T *__restrict__ fvn,
    T *__restrict__ fhat, T *__restrict__ vol, int64_t Ne, int64_t n_bc = 0, const T *__restrict__ ifc_uh = nullptr) {
  using S = Shape<D, P>;
  using TL = GradTile<D, P, T, EE>;
  constexpr int E = TL::E, Ns = S::Ns, Nf = S::Nf, Nfp = S::Nfp, NV = S::NV, NM = S::NM, NFACE = 2 * D;
  __shared__ __attribute__((aligned(16))) T lds[E * TL::LE];
  __shared__ OpsDev<T, P> ops;
  __shared__ int s_face[E * NFACE];
  __shared__ int s_nface;
  __shared__ int s_mesh[E];  // mesh of each element (free-stream data)
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (int)((Ne - e0) < E ? (Ne - e0) : E);
  // tile bases are uniform; per-thread offsets inside the tile are 32-bit
  const int32_t *nbr_t = nbr + e0 * Nf;
  const T *fnrm_t = fnrm + e0 * (D + 1) * Nf, *metric_t = metric + e0 * NM * Ns;
  using UL = UfLayout<D, P, T>;  // layout of fhat (and u_f)
  T *fvn_t = fvn + e0 * UL::EB, *fhat_t = fhat + e0 * UL::EB, *vol_t = vol + e0 * NV * Ns;
  T *lu = lds;                // [E][NV][Ns]
  T *lw = lds + E * TL::LU;   // [E][NV][Nf] u^ - u_f; then [E][Ns][D][NV] gradient; [E][D][NV][Ns] F~
  int32_t *lcode = reinterpret_cast<int32_t *>(lw + E * NV * Nf);  // [E][Nf], until the gradient phase
  T *ls = lds + E * (TL::LU + TL::LG);  // [E][D*D][Ns] (2-D): S of each thread's own point
  T *lp = ls + E * D * D * Ns;          // [E][NV][Nf] (2-D): partial common flux
  const int side = ph.side;
  // the state, the neighbour codes and the mesh indices arrive in one round trip, so the first
  // flux-point phase starts its neighbour gathers without another one; wave 0 also requests the
  // code of every face of the tile (its first flux point) for the face list below
  constexpr int KF = (E * NFACE + 63) / 64;  // faces per lane of wave 0
  int32_t fcode[KF];
  {
    TileLoad<E * NV * Ns, TL::BS, T> tu;
    TileLoad<E * Nf, TL::BS, int32_t> tc;
    tu.load(u + e0 * NV * Ns, ne * NV * Ns);
    tc.load(nbr_t, ne * Nf);
    if (threadIdx.x < 64) {
#pragma unroll
      for (int k = 0; k < KF; ++k) {
        const int fi = k * 64 + (int)threadIdx.x;
        fcode[k] = fi < ne * NFACE ? nbr_t[(uint32_t)((fi / NFACE) * Nf + (fi % NFACE) * Nfp)] : 0;
      }
    }
    const int mesh = (int)threadIdx.x < ne ? elem_mesh[e0 + threadIdx.x] : 0;
    stage_ops(ops, ops_arg);
    tu.store(lu, ne * NV * Ns);
    tc.store(lcode, ne * Nf);
    if ((int)threadIdx.x < ne) s_mesh[threadIdx.x] = mesh;
  }
  // faces of the tile ordered with those whose viscous normal flux is consumed (boundary faces,
  // and interior faces on the flux side; every flux point of a face shares its partner face and
  // its side) at the front, s_nface of them, the others behind; the flux-point phases walk this
  // order, so that the waves doing flux-side work (neighbour gather, Rusanov) are not split with
  // the others.  Built by wave 0 before the first barrier.
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const unsigned long long below = (1ull << lane) - 1ull;
    int cnt = 0, rest = 0;
#pragma unroll
    for (int k = 0; k < KF; ++k) {
      const int fi = k * 64 + lane;
      const bool in = fi < ne * NFACE;
      const int32_t code = fcode[k];
      const bool need = in && (code < 0 || side == 0 || (((code & NBR_R_BIT) != 0) == (side > 0)));
      const bool other = in && !need;
      const unsigned long long m = __ballot(need), mo = __ballot(other);
      if (need) s_face[cnt + __popcll(m & below)] = fi;
      if (other) s_face[ne * NFACE - 1 - rest - __popcll(mo & below)] = fi;
      cnt += __popcll(m);
      rest += __popcll(mo);
    }
    if (lane == 0) s_nface = cnt;
  }
  __syncthreads();
  const T wl = T(0.5) + ph.beta, wr = T(0.5) - ph.beta;     // LDG common solution: weights of u_L, u_R
  const T wlf = T(0.5) - ph.beta, wrf = T(0.5) + ph.beta;   // LDG common viscous flux: weights of F_L, F_R
  for (int pass = 0;; ++pass) {
    const int idx = flux_pass_index<TL::BS>(pass);
    if (idx >= ne * Nf) break;
    const int fc0 = s_face[idx / Nfp];
    const int el = fc0 / NFACE, fp = (fc0 % NFACE) * Nfp + idx % Nfp;
    if (side != 0 && idx >= s_nface * Nfp) {
      // one-sided LDG, the side that provides u^: u^ is its own u_f (weight exactly 1, the
      // neighbour's 0), so u^ - u_f is zero and neither the value nor the gather is needed
      for (int v = 0; v < NV; ++v) lw[(el * NV + v) * Nf + fp] = T(0);
      continue;
    }
    int base, stride, fs;
    line_of_fpt<D, P>(fp, base, stride, fs);
    const T *lv = fs ? ops.lp : ops.lm;
    T uo[NV], uh[NV];
    {
      // every line value is requested before the first product (the reads overlap)
      T val[NV][P];
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int a = 0; a < P; ++a) val[v][a] = lu[(el * NV + v) * Ns + base + a * stride];
      for (int v = 0; v < NV; ++v) {
        T s = T(0);
#pragma unroll
        for (int a = 0; a < P; ++a) s += lv[a] * val[v][a];
        uo[v] = s;
      }
    }
    const int32_t code = lcode[el * Nf + fp];
    if (code >= 0) {
      const int32_t c = code & (NBR_R_BIT - 1);
      const int64_t e2 = c / Nf;
      const int f2 = c % Nf;
      const bool isR = (code & NBR_R_BIT) != 0;
      const T wn = isR ? wl : wr;  // weight of the neighbour's value; zero on the one-sided LDG's other side
      T un[NV];
      if (wn != T(0)) {  // one branch around the point's NV loads, so that they issue together
        const T *up = uf + UfLayout<D, P, T>::at(e2, 0, f2);
        for (int v = 0; v < NV; ++v) un[v] = up[v * UfLayout<D, P, T>::VS];
      } else {
        for (int v = 0; v < NV; ++v) un[v] = T(0);
      }
      for (int v = 0; v < NV; ++v) uh[v] = isR ? wl * un[v] + wr * uo[v] : wl * uo[v] + wr * un[v];
      if (side != 0 && wn != T(0)) {
        // flux side of a one-sided pair: inviscid common flux along n_L plus the penalty, x |N|,
        // into this point's fhat (2-D: its LDS slot); the flux-point phase adds the viscous part
        T n[D], F[NV];
        for (int j = 0; j < D; ++j) n[j] = fnrm_t[(uint32_t)((el * (D + 1) + j) * Nf + fp)];
        const T mag = fnrm_t[(uint32_t)((el * (D + 1) + D) * Nf + fp)];
        if (isR) {
          for (int j = 0; j < D; ++j) n[j] = -n[j];  // n_L
          rusanov<D>(un, uo, n, ph.gamma, ph.gm1, F);
          for (int v = 0; v < NV; ++v) F[v] = (F[v] + ph.tau * (un[v] - uo[v])) * mag;
        } else {
          rusanov<D>(uo, un, n, ph.gamma, ph.gm1, F);
          for (int v = 0; v < NV; ++v) F[v] = (F[v] + ph.tau * (uo[v] - un[v])) * mag;
        }
        if constexpr (TL::KEEP2D) {
          for (int v = 0; v < NV; ++v) lp[(el * NV + v) * Nf + fp] = F[v];
        } else {
          T *fo = fhat_t + (uint32_t)UL::point(el, fp);
          for (int v = 0; v < NV; ++v) fo[v * UL::VS] = F[v];
        }
      }
    } else {
      const int64_t b = -(int64_t)code - 1;
      T n[D];
      for (int j = 0; j < D; ++j) n[j] = bnrm[b * (D + 1) + j];
      const bool wall = b < n_wall;
      const bool mortar = MORTAR && b >= n_bc;
      if (mortar) {
        for (int v = 0; v < NV; ++v) uh[v] = ifc_uh[(b - n_bc) * NV + v];
      } else if (wall) {
        wall_state<D>(uo, uh);
      } else {
        farfield<D>(uo, n, flow[s_mesh[el]], ph.gamma, ph.gm1, uh);
      }
      if (side != 0 && !mortar) {
        // boundary flux, inviscid part: Rusanov against the ghost (wall reflection / far-field state)
        T ug[NV], F[NV];
        if (wall) {
          ug[0] = uo[0];
          for (int j = 0; j < D; ++j) ug[1 + j] = -uo[1 + j];
          ug[D + 1] = uo[D + 1];
        } else {
          for (int v = 0; v < NV; ++v) ug[v] = uh[v];
        }
        rusanov<D>(uo, ug, n, ph.gamma, ph.gm1, F);
        const T mag = bnrm[b * (D + 1) + D];
        if constexpr (TL::KEEP2D) {
          for (int v = 0; v < NV; ++v) lp[(el * NV + v) * Nf + fp] = F[v] * mag;
        } else {
          T *fo = fhat_t + (uint32_t)UL::point(el, fp);
          for (int v = 0; v < NV; ++v) fo[v * UL::VS] = F[v] * mag;
        }
      }
    }
    for (int v = 0; v < NV; ++v) lw[(el * NV + v) * Nf + fp] = uh[v] - uo[v];
  }
  __syncthreads();
  const int el = threadIdx.x / Ns, i = threadIdx.x % Ns;
  const bool act = el < ne;
  // corrected physical gradient at the own solution point
  T gx[D][NV];
  if (act) {
    T Sm[D][D];
    for (int k = 0; k < D; ++k)
      for (int j = 0; j < D; ++j) Sm[k][j] = metric_t[(uint32_t)((el * NM + k * D + j) * Ns + i)];
    const T invJ = metric_t[(uint32_t)((el * NM + D * D) * Ns + i)];
    if constexpr (TL::KEEP2D)
      for (int k = 0; k < D; ++k)
        for (int j = 0; j < D; ++j) ls[(el * D * D + k * D + j) * Ns + i] = Sm[k][j];
    for (int j = 0; j < D; ++j)
      for (int v = 0; v < NV; ++v) gx[j][v] = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      int base, stride, ik, t;
      line_of_sol<D, P>(i, k, base, stride, ik, t);
      const T cm = -ops.gm[ik], cp = ops.gp[ik];
      T Sk[D];  // row k selected without dynamic indexing into a private array
      for (int j = 0; j < D; ++j) {
        Sk[j] = Sm[0][j];
        for (int q = 1; q < D; ++q)
          if (k == q) Sk[j] = Sm[q][j];
      }
      for (int v = 0; v < NV; ++v) {
        const T *lin = lu + (el * NV + v) * Ns + base;
        T s = T(0);
#pragma unroll
        for (int a = 0; a < P; ++a) s += ops.D[ik * P + a] * lin[a * stride];
        const T *ld = lw + (el * NV + v) * Nf;
        s += cm * ld[(2 * k) * Nfp + t] + cp * ld[(2 * k + 1) * Nfp + t];
        for (int j = 0; j < D; ++j) gx[j][v] += Sk[j] * s;
      }
    }
    for (int j = 0; j < D; ++j)
      for (int v = 0; v < NV; ++v) gx[j][v] *= invJ;
  }
  __syncthreads();
  // gradient point-major, [E][Ns][D][NV]: the flux-point interpolation reads the D*NV values of
  // one line point at constant offsets from one address
  if (act)
    for (int j = 0; j < D; ++j)
      for (int v = 0; v < NV; ++v) lw[(el * Ns + i) * (D * NV) + j * NV + v] = gx[j][v];
  __syncthreads();
  // Flux points of the listed faces: viscous normal flux fvn = F_vis(u_f, M0 grad_x u) . n_out.
  // Two-sided LDG: stored for the face kernel.  One-sided LDG: this point's side alone supplies
  // the viscous part of the common flux and holds both states, so the first phase already put
  // the inviscid part and the penalty (x |N|) into its fhat (2-D: LDS); here the viscous part is
  // added and the finished common flux goes to both sides of the pair (boundary points: own side
  // only).
  // fvn is stored on boundary points in both modes (wall-force integral).
  const int nfc = s_nface;
  for (int pass = 0;; ++pass) {
    const int idx = flux_pass_index<TL::BS>(pass);
    if (idx >= nfc * Nfp) break;
    const int fc = s_face[idx / Nfp];
    const int elf = fc / NFACE, fp = (fc % NFACE) * Nfp + idx % Nfp;
    int base, stride, fs;
    line_of_fpt<D, P>(fp, base, stride, fs);
    const T *lv = fs ? ops.lp : ops.lm;
    T uo[NV], st[NV], n[D];
    {
      T val[NV][P];  // every line value requested before the first product
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int a = 0; a < P; ++a) val[v][a] = lu[(elf * NV + v) * Ns + base + a * stride];
      for (int v = 0; v < NV; ++v) {
        T s = T(0);
#pragma unroll
        for (int a = 0; a < P; ++a) s += lv[a] * val[v][a];
        uo[v] = s;
      }
    }
    for (int j = 0; j < D; ++j) n[j] = fnrm_t[(uint32_t)((elf * (D + 1) + j) * Nf + fp)];
    const int32_t code = nbr_t[(uint32_t)(elf * Nf + fp)];
    const FlowDev<T> &fl = flow[s_mesh[elf]];
    // the common-flux partial of the first phase (2-D: from LDS) and |N| are requested with the
    // other loads
    T *fo = fhat_t + (uint32_t)UL::point(elf, fp);
    T fprev[NV], mag = T(0);
    if (side != 0) {
      mag = fnrm_t[(uint32_t)((elf * (D + 1) + D) * Nf + fp)];
      for (int v = 0; v < NV; ++v) fprev[v] = TL::KEEP2D ? lp[(elf * NV + v) * Nf + fp] : fo[v * UL::VS];
    }
    bool heat = true, wall = false, mortar = false;
    if (code < 0) {
      const int64_t b = -(int64_t)code - 1;
      wall = b < n_wall;
      mortar = MORTAR && b >= n_bc;
      if (mortar) {
        for (int v = 0; v < NV; ++v) st[v] = uo[v];
      } else if (wall) {
        wall_state<D>(uo, st);
        heat = false;
      } else {
        farfield<D>(uo, n, fl, ph.gamma, ph.gm1, st);
      }
    } else {
      for (int v = 0; v < NV; ++v) st[v] = uo[v];
    }
    const T *lge = lw + (elf * Ns + base) * (D * NV);
    auto gdir = [&](int d, T *gd) {
      for (int v = 0; v < NV; ++v) gd[v] = T(0);
#pragma unroll
      for (int a = 0; a < P; ++a) {
        const T *row = lge + a * stride * (D * NV) + d * NV;
        for (int v = 0; v < NV; ++v) gd[v] += lv[a] * row[v];
      }
    };
    T fv[NV];
    fvis_normal_stream<D>(st, gdir, n, fl.mu, ph, heat, fv);
    if (side == 0 || code < 0)
      for (int v = 0; v < NV; ++v) fvn_t[(fo - fhat_t) + v * UL::VS] = fv[v];  // same offset as fo
    if (side == 0) continue;
    // complete the common flux started in the first phase (same workgroup, ordered by the barriers)
    if (code < 0) {
      if (!mortar)
        for (int v = 0; v < NV; ++v) fo[v * UL::VS] = fprev[v] - fv[v] * mag;
    } else {
      const int32_t c = code & (NBR_R_BIT - 1);
      T *fq = fhat + UL::point((int64_t)(c / Nf), c % Nf);
      if (code & NBR_R_BIT) {  // F^ . n_L = ... + (1/2 + b) fvn_R
        for (int v = 0; v < NV; ++v) {
          const T t = fprev[v] + wrf * fv[v] * mag;
          fo[v * UL::VS] = -t;
          fq[v * UL::VS] = t;
        }
      } else {                 // F^ . n_L = ... - (1/2 - b) fvn_L
        for (int v = 0; v < NV; ++v) {
          const T t = fprev[v] - wlf * fv[v] * mag;
          fo[v * UL::VS] = t;
          fq[v * UL::VS] = -t;
        }
      }
    }
  }
  // transformed flux F~_k = S_k . (F_inv - F_vis) at the own solution point, from the gradient
  // held in LDS (no transformed flux is live in registers through the flux-point phase)
  T ft[D][NV];
  if (act) {
    T uv[NV], g[D * NV];
    for (int v = 0; v < NV; ++v) uv[v] = lu[(el * NV + v) * Ns + i];
    for (int c = 0; c < D * NV; ++c) g[c] = lw[(el * Ns + i) * (D * NV) + c];
    Visc<D, T> vs;
    visc_state<D>(uv, g, flow[s_mesh[el]].mu, ph, true, vs);
    for (int k = 0; k < D; ++k) {
      T Sk[D], fi[NV], fv[NV];
      for (int j = 0; j < D; ++j)
        Sk[j] = TL::KEEP2D ? ls[(el * D * D + k * D + j) * Ns + i]                  // own LDS copy
                           : metric_t[(uint32_t)((el * NM + k * D + j) * Ns + i)];  // second read
      finv_dot<D>(uv, Sk, ph.gm1, fi);
      fvis_dot<D>(vs, Sk, fv);
      for (int v = 0; v < NV; ++v) ft[k][v] = fi[v] - fv[v];
    }
  }
  __syncthreads();
  if (act)
    for (int k = 0; k < D; ++k)
      for (int v = 0; v < NV; ++v) lw[((el * D + k) * NV + v) * Ns + i] = ft[k][v];
  __syncthreads();
  if constexpr (MFMA_DIV) {
    mfma_divergence<D, P, TL::BS>(lw, lu, ops.Dt, ne, E);
    if (act)
      for (int v = 0; v < NV; ++v) vol_t[(uint32_t)((el * NV + v) * Ns + i)] = lu[(el * NV + v) * Ns + i];
    return;
  }
  if (act) {
    T accv[NV];
    for (int v = 0; v < NV; ++v) accv[v] = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      int base, stride, ik, t;
      line_of_sol<D, P>(i, k, base, stride, ik, t);
      const T *dt = ops.Dt + ik * P;
      for (int v = 0; v < NV; ++v) {
        const T *lin = lw + ((el * D + k) * NV + v) * Ns + base;
        T ds = T(0);
#pragma unroll
        for (int a = 0; a < P; ++a) ds += dt[a] * lin[a * stride];
        accv[v] += ds;
      }
    }
    for (int v = 0; v < NV; ++v) vol_t[(uint32_t)((el * NV + v) * Ns + i)] = accv[v];
  }
}

// RK epilogue arguments
template <typename T>
struct RKArgs {
  T *r_out;          // residual output (rhs mode) or nullptr
  T *u0;             // base state (read; written on the last stage)
  T *acc;            // RK accumulator
  T *ustage;         // next stage state (not last)
  const double *dt;  // per mesh
  T cA, cB;          // u_next = u0 + cA dt R ; acc += cB dt R
  int first, last;
  T *uf_next;        // flux-point values of the new stage state, or nullptr
  const uint8_t *uf_faces;  // faces whose flux-point values are written (bit f per element)
  T *ustage_copy;    // optional second copy of the new stage state (adjoint recording)
  T *u0_copy;        // optional copy of the base state (adjoint recording, first stage)
  T *r_copy;         // optional copy of this stage's residual (adjoint recording)
};

// what the RK epilogue reads at (e, i): requested with the kernel's other loads so that their
// latency is shared
template <typename T, int NV>
struct RKIn {
  T u0[NV], acc[NV];
  int mesh;
};

template <int D, int P, typename T>
__device__ __forceinline__ void rk_prefetch(int64_t e, int i, const RKArgs<T> &rk,
                                            const int32_t *__restrict__ elem_mesh, RKIn<T, Shape<D, P>::NV> &in) {
  using S = Shape<D, P>;
  constexpr int NV = S::NV, Ns = S::Ns;
  in.mesh = 0;
  if (rk.r_out) return;
  in.mesh = elem_mesh[e];
  for (int v = 0; v < NV; ++v) {
    const int64_t o = (e * NV + v) * Ns + i;
    in.u0[v] = rk.u0[o];
    in.acc[v] = rk.first ? T(0) : rk.acc[o];
  }
}

// shared epilogue: R at (el, i) for all variables -> rhs output or RK update; the new stage
// state goes to `w` (for the flux-point values of the next stage)
template <int D, int P, typename T>
__device__ __forceinline__ void rk_epilogue(const T *R, int64_t e, int i, const RKArgs<T> &rk,
                                            const RKIn<T, Shape<D, P>::NV> &in, T *w) {
  using S = Shape<D, P>;
  constexpr int NV = S::NV, Ns = S::Ns;
  if (rk.r_out) {
    for (int v = 0; v < NV; ++v) rk.r_out[(e * NV + v) * Ns + i] = R[v];
    return;
  }
  const T dt = (T)rk.dt[in.mesh];
  for (int v = 0; v < NV; ++v) {
    const int64_t o = (e * NV + v) * Ns + i;
    if (rk.r_copy) rk.r_copy[o] = R[v];
    const T a = in.acc[v];
    const T u0 = in.u0[v];
    if (rk.u0_copy) rk.u0_copy[o] = u0;
    if (!rk.last) {
      rk.acc[o] = a + rk.cB * dt * R[v];
      w[v] = u0 + rk.cA * dt * R[v];
      rk.ustage[o] = w[v];
      if (rk.ustage_copy) rk.ustage_copy[o] = w[v];
    } else {
      w[v] = u0 + (a + rk.cB * dt * R[v]);
      rk.u0[o] = w[v];
    }
  }
}

// u_f = M0 u of a tile from its state in LDS ([E][NV][Ns]).  Face-blocked layout: the faces
// flagged in faces[el] (bit f; an LDS copy of the tile's entries), each block one run of whole
// lines; otherwise every value, contiguously
template <int D, int P, typename T>
__device__ __forceinline__ void tile_interp(const T *lw, int ne, const OpsDev<T, P> &ops, T *uf_tile,
                                            const uint8_t *faces) {
  using S = Shape<D, P>;
  using L = UfLayout<D, P, T>;
  constexpr int NV = S::NV, Ns = S::Ns, Nf = S::Nf, Nfp = S::Nfp, FB = L::FB, NFACE = L::NFACE;
  if constexpr (L::SKIP) {
    for (int idx = threadIdx.x; idx < ne * NFACE * FB; idx += blockDim.x) {
      const int ef = idx / FB, r = idx % FB;  // ef = element * NFACE + face
      const int el = ef / NFACE, f = ef % NFACE;
      if (!((faces[el] >> f) & 1)) continue;
      const int v = r / Nfp, fp = f * Nfp + r % Nfp;
      int base, stride, side;
      line_of_fpt<D, P>(fp, base, stride, side);
      const T *lv = side ? ops.lp : ops.lm;
      const T *lin = lw + (el * NV + v) * Ns + base;
      T s = T(0);
#pragma unroll
      for (int a = 0; a < P; ++a) s += lv[a] * lin[a * stride];
      uf_tile[ef * L::FS + r] = s;
    }
  } else {
    for (int idx = threadIdx.x; idx < ne * NV * Nf; idx += blockDim.x) {
      const int fp = idx % Nf, rest = idx / Nf;  // rest = element * NV + v
      int base, stride, side;
      line_of_fpt<D, P>(fp, base, stride, side);
      const T *lv = side ? ops.lp : ops.lm;
      const T *lin = lw + rest * Ns + base;
      T s = T(0);
#pragma unroll
      for (int a = 0; a < P; ++a) s += lv[a] * lin[a * stride];
      uf_tile[idx] = s;
    }
  }
}

// u_f = M0 u on the flagged faces, E elements per workgroup: the state tile is staged in LDS
// (contiguous loads, one round trip) and every flux-point value is written once
template <int D, int P, typename T>
__global__ __launch_bounds__((DivTile<D, P, T>::BS)) void k_interp(const T *__restrict__ u, T *__restrict__ uf,
                                                                   const uint8_t *__restrict__ uf_faces,
                                                                   OpsDev<T, P> ops_arg, int64_t Ne) {
  using S = Shape<D, P>;
  using TL = DivTile<D, P, T>;
  constexpr int E = TL::E, NV = S::NV, Ns = S::Ns;
  __shared__ __attribute__((aligned(16))) T lu[E * NV * Ns];
  __shared__ OpsDev<T, P> ops;
  __shared__ uint8_t s_faces[E];
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (int)((Ne - e0) < E ? (Ne - e0) : E);
  TileLoad<E * NV * Ns, TL::BS, T> tu;
  tu.load(u + e0 * NV * Ns, ne * NV * Ns);
  const uint8_t fmask = (UfLayout<D, P, T>::SKIP && (int)threadIdx.x < ne) ? uf_faces[e0 + threadIdx.x] : 0;
  stage_ops(ops, ops_arg);
  if ((int)threadIdx.x < ne) s_faces[threadIdx.x] = fmask;
  tu.store(lu, ne * NV * Ns);
  __syncthreads();
  tile_interp<D, P>(lu, ne, ops, uf + e0 * UfLayout<D, P, T>::EB, s_faces);
}

// NS: R = -(1/J)(vol + Lift F^), RK update, u_f of the new stage state
template <int D, int P, typename T, int EE>
__device__ __forceinline__ void div_rk_body(const T *__restrict__ vol, const T *__restrict__ fhat,
                                            const T *__restrict__ metric, const int32_t *__restrict__ elem_mesh,
                                            const OpsDev<T, P> &ops_arg, const RKArgs<T> &rk, int64_t Ne) {
  using S = Shape<D, P>;
  using TL = DivTile<D, P, T, EE>;
  constexpr int E = TL::E, Ns = S::Ns, NV = S::NV, NM = S::NM;
  __shared__ __attribute__((aligned(16))) T lds[E * TL::LE];
  __shared__ OpsDev<T, P> ops;
  __shared__ uint8_t s_faces[E];
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (int)((Ne - e0) < E ? (Ne - e0) : E);
  const int el = threadIdx.x / Ns, i = threadIdx.x % Ns;
  const bool act = el < ne;
  const int64_t e = e0 + el;
  // the common-flux tile, this point's volume term, 1/J, the RK inputs and the tile's u_f face
  // flags in one round trip
  using UL = UfLayout<D, P, T>;
  TileLoad<E * UL::EB, TL::BS, T> tf;
  tf.load(fhat + e0 * UL::EB, ne * UL::EB);
  const uint8_t fmask = (UL::SKIP && rk.uf_next && (int)threadIdx.x < ne) ? rk.uf_faces[e0 + threadIdx.x] : 0;
  T R[NV], invJ = T(0);
  RKIn<T, NV> in;
  if (act) {
    invJ = metric[(e * NM + D * D) * Ns + i];
    for (int v = 0; v < NV; ++v) R[v] = vol[(e * NV + v) * Ns + i];
    rk_prefetch<D, P>(e, i, rk, elem_mesh, in);
  }
  stage_ops(ops, ops_arg);
  tf.store(lds, ne * UL::EB);
  if ((int)threadIdx.x < ne) s_faces[threadIdx.x] = fmask;
  __syncthreads();
  T w[NV];
  if (act) {
    for (int k = 0; k < D; ++k) {
      int base, stride, ik, t;
      line_of_sol<D, P>(i, k, base, stride, ik, t);
      const T gm = ops.gm[ik], gp = ops.gp[ik];
      for (int v = 0; v < NV; ++v) {
        const T *lf = lds + el * UL::EB + v * UL::VS;
        R[v] += gm * lf[(2 * k) * UL::FST + t] + gp * lf[(2 * k + 1) * UL::FST + t];
      }
    }
    for (int v = 0; v < NV; ++v) R[v] = -invJ * R[v];
    rk_epilogue<D, P>(R, e, i, rk, in, w);
  }
  if (rk.uf_next) {
    __syncthreads();
    if (act)
      for (int v = 0; v < NV; ++v) lds[(el * NV + v) * Ns + i] = w[v];
    __syncthreads();
    tile_interp<D, P>(lds, ne, ops, rk.uf_next + e0 * UfLayout<D, P, T>::EB, s_faces);
  }
}

// the lifting + RK kernel with the compiler's register budget, and with a waves-per-SIMD launch
// bound WW (an autotuner candidate); same body
template <int D, int P, typename T, int EE>
__global__ __launch_bounds__((DivTile<D, P, T, EE>::BS)) void k_div_rk(const T *__restrict__ vol,
                                                                const T *__restrict__ fhat,
                                                                const T *__restrict__ metric,
                                                                const int32_t *__restrict__ elem_mesh,
                                                                OpsDev<T, P> ops_arg, RKArgs<T> rk, int64_t Ne) {
  div_rk_body<D, P, T, EE>(vol, fhat, metric, elem_mesh, ops_arg, rk, Ne);
}
template <int D, int P, typename T, int EE, int WW>
__global__ __launch_bounds__((DivTile<D, P, T, EE>::BS), WW) void k_div_rk_w(const T *__restrict__ vol,
                                                                      const T *__restrict__ fhat,
                                                                      const T *__restrict__ metric,
                                                                      const int32_t *__restrict__ elem_mesh,
                                                                      OpsDev<T, P> ops_arg, RKArgs<T> rk,
                                                                      int64_t Ne) {
  div_rk_body<D, P, T, EE>(vol, fhat, metric, elem_mesh, ops_arg, rk, Ne);
}

// Euler: F~ at solution points, volume divergence with interior correction, lifting of the
// common flux, RK update and u_f of the new stage state, in one kernel
template <int D, int P, typename T, int EE>
__device__ __forceinline__ void euler_vol_rk_body(
    const T *u,  // may alias rk.ustage: every thread reads its own point before writing it
    const T *__restrict__ fhat, const T *__restrict__ metric,
    const int32_t *__restrict__ elem_mesh, const OpsDev<T, P> &ops_arg, const PhysDev<T> &ph, const RKArgs<T> &rk,
    int64_t Ne) {
  using S = Shape<D, P>;
  using TL = EulerTile<D, P, T, EE>;
  constexpr int E = TL::E, Ns = S::Ns, NV = S::NV, NM = S::NM;
  __shared__ __attribute__((aligned(16))) T lds[E * TL::LE];
  __shared__ OpsDev<T, P> ops;
  __shared__ uint8_t s_faces[E];
  T *lF = lds;                  // [E][D][NV][Ns]
  T *lf = lds + E * D * NV * Ns;  // common-flux tile, layout of fhat
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (int)((Ne - e0) < E ? (Ne - e0) : E);
  const int el = threadIdx.x / Ns, i = threadIdx.x % Ns;
  const bool act = el < ne;
  const int64_t e = e0 + el;
  // the common-flux tile, this point's state and metric terms, the RK inputs and the tile's u_f
  // face flags in one round trip
  using UL = UfLayout<D, P, T>;
  TileLoad<E * UL::EB, TL::BS, T> tf;
  tf.load(fhat + e0 * UL::EB, ne * UL::EB);
  const uint8_t fmask = (UL::SKIP && rk.uf_next && (int)threadIdx.x < ne) ? rk.uf_faces[e0 + threadIdx.x] : 0;
  T invJ = T(0), uv[NV], Sm[D][D];
  RKIn<T, NV> in;
  if (act) {
    for (int v = 0; v < NV; ++v) uv[v] = u[(e * NV + v) * Ns + i];
    for (int k = 0; k < D; ++k)
      for (int j = 0; j < D; ++j) Sm[k][j] = metric[(e * NM + k * D + j) * Ns + i];
    invJ = metric[(e * NM + D * D) * Ns + i];
    rk_prefetch<D, P>(e, i, rk, elem_mesh, in);
  }
  stage_ops(ops, ops_arg);
  tf.store(lf, ne * UL::EB);
  if ((int)threadIdx.x < ne) s_faces[threadIdx.x] = fmask;
  if (act) {
    for (int k = 0; k < D; ++k) {
      T fi[NV];
      finv_dot<D>(uv, Sm[k], ph.gm1, fi);
      for (int v = 0; v < NV; ++v) lF[((el * D + k) * NV + v) * Ns + i] = fi[v];
    }
  }
  __syncthreads();
  T w[NV];
  if (act) {
    T R[NV];
    for (int v = 0; v < NV; ++v) {
      T accv = T(0);
#pragma unroll 1
      for (int k = 0; k < D; ++k) {
        int base, stride, ik, t;
        line_of_sol<D, P>(i, k, base, stride, ik, t);
        const T *lin = lF + ((el * D + k) * NV + v) * Ns + base;
        T ds = T(0);
#pragma unroll
        for (int a = 0; a < P; ++a) ds += ops.Dt[ik * P + a] * lin[a * stride];
        const T *lfv = lf + el * UL::EB + v * UL::VS;
        accv += ds + ops.gm[ik] * lfv[(2 * k) * UL::FST + t] + ops.gp[ik] * lfv[(2 * k + 1) * UL::FST + t];
      }
      R[v] = -invJ * accv;
    }
    rk_epilogue<D, P>(R, e, i, rk, in, w);
  }
  if (rk.uf_next) {
    __syncthreads();
    if (act)
      for (int v = 0; v < NV; ++v) lds[(el * NV + v) * Ns + i] = w[v];
    __syncthreads();
    tile_interp<D, P>(lds, ne, ops, rk.uf_next + e0 * UfLayout<D, P, T>::EB, s_faces);
  }
}

template <int D, int P, typename T, int EE>
__global__ __launch_bounds__((EulerTile<D, P, T, EE>::BS)) void k_euler_vol_rk(
    const T *u, const T *__restrict__ fhat, const T *__restrict__ metric, const int32_t *__restrict__ elem_mesh,
    OpsDev<T, P> ops_arg, PhysDev<T> ph, RKArgs<T> rk, int64_t Ne) {
  euler_vol_rk_body<D, P, T, EE>(u, fhat, metric, elem_mesh, ops_arg, ph, rk, Ne);
}
template <int D, int P, typename T, int EE, int WW>
__global__ __launch_bounds__((EulerTile<D, P, T, EE>::BS), WW) void k_euler_vol_rk_w(
    const T *u, const T *__restrict__ fhat, const T *__restrict__ metric, const int32_t *__restrict__ elem_mesh,
    OpsDev<T, P> ops_arg, PhysDev<T> ph, RKArgs<T> rk, int64_t Ne) {
  euler_vol_rk_body<D, P, T, EE>(u, fhat, metric, elem_mesh, ops_arg, ph, rk, Ne);
}

// probe pressure samples (FP64): one workgroup per probe, the weighted sum over the element's
// solution points reduced in a fixed tree.  count[0] is the sample index, count[1] a ticket: each
// workgroup reads the index, stores its sample, then takes a ticket, and the last one advances
// the index (every workgroup has read it by then) and clears the ticket
constexpr int PROBE_BS = 128;  // >= Ns for p <= 4
template <int D, int P, typename T>
__global__ __launch_bounds__(PROBE_BS) void k_probe(const T *__restrict__ u, const int64_t *__restrict__ pelem,
                                                    const double *__restrict__ pw, const double *__restrict__ pinf,
                                                    double gm1, double *series, int cap, double *sums,
                                                    unsigned long long *count, int *nonfinite) {
  using S = Shape<D, P>;
  constexpr int NV = S::NV, Ns = S::Ns;
  static_assert(Ns <= PROBE_BS, "one solution point per thread");
  __shared__ double red[NV][PROBE_BS];
  const int a = blockIdx.x, i = threadIdx.x;
  const int64_t e = pelem[a];
  const double w = i < Ns ? pw[(int64_t)a * Ns + i] : 0.0;
  for (int v = 0; v < NV; ++v) red[v][i] = i < Ns ? w * (double)u[(e * NV + v) * Ns + i] : 0.0;
  __syncthreads();
  for (int st = PROBE_BS / 2; st > 0; st >>= 1) {
    if (i < st)
      for (int v = 0; v < NV; ++v) red[v][i] += red[v][i + st];
    __syncthreads();
  }
  if (i == 0) {
    const unsigned long long n = *count;
    double ke = 0.0;
    for (int j = 0; j < D; ++j) ke += red[1 + j][0] * red[1 + j][0];
    const double p = gm1 * (red[D + 1][0] - 0.5 * ke / red[0][0]);
    if (n < (unsigned long long)cap) series[(int64_t)a * cap + (int64_t)n] = p;
    const double dp = p - pinf[a];
    sums[2 * a] += dp;
    sums[2 * a + 1] += dp * dp;
    if (!isfinite(p)) *nonfinite = 1;
    __threadfence();
    if (atomicAdd(&count[1], 1ull) == (unsigned long long)(gridDim.x - 1)) {
      count[0] = n + 1;
      count[1] = 0ull;
    }
  }
}

// the sample index of a sample without probes (forces only)
__global__ void k_probe_count(unsigned long long *count) {
  if (threadIdx.x == 0) count[0] += 1;
}

// wall force per mesh (FP64): sum over wall flux points of w |N| (p n - tau n), tau n being the
// momentum part of the wall viscous normal flux.  Workgroup (chunk c, mesh m) sums the chunk's
// WALL_CHUNK points in a fixed tree into partial[m][c]; k_wall_force_sum adds the chunks of a mesh
// in order (deterministic, no atomics).
template <int D, int P, typename T>
__global__ __launch_bounds__(WALL_CHUNK) void k_wall_force(const T *__restrict__ uf, const T *__restrict__ fvn,
                                                           const int32_t *__restrict__ bnd,
                                                           const T *__restrict__ bnrm, const double *__restrict__ bw,
                                                           const int64_t *__restrict__ wall_begin, PhysDev<T> ph,
                                                           int nchunk, double *__restrict__ partial) {
  using S = Shape<D, P>;
  constexpr int NV = S::NV, Nf = S::Nf;
  __shared__ double red[WALL_CHUNK][D];
  const int m = blockIdx.y, c = blockIdx.x;
  const int64_t b = wall_begin[m] + (int64_t)c * WALL_CHUNK + threadIdx.x;
  double f[D];
  for (int j = 0; j < D; ++j) f[j] = 0.0;
  if (b < wall_begin[m + 1]) {
    const int32_t code = bnd[b];
    const int64_t e = code / Nf;
    const int fp = code % Nf;
    T uB[NV];
    for (int v = 0; v < NV; ++v) uB[v] = uf[UfLayout<D, P, T>::at(e, v, fp)];
    T rho, vel[D], p;
    primitives<D>(uB, ph.gm1, rho, vel, p);
    const double wm = bw[b] * (double)bnrm[b * (D + 1) + D];
    for (int j = 0; j < D; ++j)
      f[j] = wm * ((double)p * (double)bnrm[b * (D + 1) + j] - (double)fvn[UfLayout<D, P, T>::at(e, 1 + j, fp)]);
  }
  for (int j = 0; j < D; ++j) red[threadIdx.x][j] = f[j];
  __syncthreads();
  for (int st = WALL_CHUNK / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int j = 0; j < D; ++j) red[threadIdx.x][j] += red[threadIdx.x + st][j];
    __syncthreads();
  }
  if (threadIdx.x < D) partial[((int64_t)m * nchunk + c) * D + threadIdx.x] = red[0][threadIdx.x];
}

// lane l of the 64 sums chunks l, l + 64, ... in order, then a fixed tree over the lanes
template <int D>
__global__ __launch_bounds__(64) void k_wall_force_sum(const double *__restrict__ partial, int nchunk,
                                                       double *force_acc) {
  __shared__ double red[64][D];
  const int m = blockIdx.x, l = threadIdx.x;
  double s[D];
  for (int j = 0; j < D; ++j) s[j] = 0.0;
  for (int c = l; c < nchunk; c += 64)
    for (int j = 0; j < D; ++j) s[j] += partial[((int64_t)m * nchunk + c) * D + j];
  for (int j = 0; j < D; ++j) red[l][j] = s[j];
  __syncthreads();
  for (int st = 32; st > 0; st >>= 1) {
    if (l < st)
      for (int j = 0; j < D; ++j) red[l][j] += red[l + st][j];
    __syncthreads();
  }
  if (l < D) force_acc[m * D + l] += red[0][l];
}

// adjoint of the probe samples: u_bar += sum_a p_bar[a] dp_a/du.  With x_bar: the probe is fixed
// in physical space, so its reference coordinates xi move with its element's nodes
// (d xi / d X_n = -A^{-1} phi_n, tabulated per probe), and x_bar += p_bar (dp/dxi) (d xi / d X).
// k_probe_vjp_coef (one workgroup per probe, fixed reduction trees) forms each probe's
// coefficients p_bar dp/du_v and p_bar dp/dxi_k; k_probe_vjp_scatter (one workgroup) adds them into
// u_bar and x_bar probe by probe, so probes that share an element or nodes add in a fixed order.
// One probe: k_probe_vjp_one does both in one workgroup (one launch instead of two).

// coefficients of probe a into out[NV + D] (thread 0 writes; every thread of the workgroup calls)
template <int D, int P, typename T>
__device__ __forceinline__ void probe_vjp_coef_body(const T *__restrict__ u, const int64_t *__restrict__ pelem,
                                                    const double *__restrict__ pw, const double *__restrict__ pdw,
                                                    double gm1, const double *__restrict__ pbar, bool geo, int a,
                                                    double *out) {
  using S = Shape<D, P>;
  constexpr int NV = S::NV, Ns = S::Ns;
  __shared__ double red[NV][PROBE_BS];
  __shared__ double dpdu[NV];
  const int i = threadIdx.x;
  const int64_t e = pelem[a];
  double uv[NV];
  for (int v = 0; v < NV; ++v) uv[v] = i < Ns ? (double)u[(e * NV + v) * Ns + i] : 0.0;
  const double w = i < Ns ? pw[(int64_t)a * Ns + i] : 0.0;
  for (int v = 0; v < NV; ++v) red[v][i] = w * uv[v];
  __syncthreads();
  for (int st = PROBE_BS / 2; st > 0; st >>= 1) {
    if (i < st)
      for (int v = 0; v < NV; ++v) red[v][i] += red[v][i + st];
    __syncthreads();
  }
  const double pb = pbar[a];
  if (i == 0) {
    // p = (gamma-1)(E - |m|^2 / (2 rho)) at the interpolated state
    double m2 = 0.0;
    for (int j = 0; j < D; ++j) m2 += red[1 + j][0] * red[1 + j][0];
    dpdu[0] = gm1 * 0.5 * m2 / (red[0][0] * red[0][0]);
    for (int j = 0; j < D; ++j) dpdu[1 + j] = -gm1 * red[1 + j][0] / red[0][0];
    dpdu[D + 1] = gm1;
    for (int v = 0; v < NV; ++v) out[v] = pb * dpdu[v];
  }
  if (!geo) return;
  __syncthreads();
  // dp/dxi_k = sum_v dp/du_v sum_i (d w_i / d xi_k) u_{v,i}
  double t[D];
  for (int k = 0; k < D; ++k) {
    t[k] = 0.0;
    if (i < Ns)
      for (int v = 0; v < NV; ++v) t[k] += dpdu[v] * pdw[((int64_t)a * D + k) * Ns + i] * uv[v];
  }
  __syncthreads();
  for (int k = 0; k < D; ++k) red[k][i] = t[k];
  __syncthreads();
  for (int st = PROBE_BS / 2; st > 0; st >>= 1) {
    if (i < st)
      for (int k = 0; k < D; ++k) red[k][i] += red[k][i + st];
    __syncthreads();
  }
  if (i == 0)
    for (int k = 0; k < D; ++k) out[NV + k] = pb * red[k][0];
}

// probe a's coefficients c added into u_bar and (xbar != nullptr) x_bar by one workgroup
template <int D, int P, typename T>
__device__ __forceinline__ void probe_vjp_scatter_one(const int64_t *__restrict__ pelem, const double *__restrict__ pw,
                                                      const double *__restrict__ pdxi,
                                                      const int64_t *__restrict__ pnodes, int nn, int a,
                                                      const double *c, T *ubar, double *xbar) {
  using S = Shape<D, P>;
  constexpr int NV = S::NV, Ns = S::Ns;
  const int64_t e = pelem[a];
  for (int idx = threadIdx.x; idx < NV * Ns; idx += blockDim.x) {
    const int v = idx / Ns, i = idx % Ns;
    ubar[(e * NV + v) * Ns + i] += (T)(c[v] * pw[(int64_t)a * Ns + i]);
  }
  if (xbar)
    for (int idx = threadIdx.x; idx < nn * D; idx += blockDim.x) {
      const int n = idx / D, j = idx % D;
      double sx = 0.0;
      for (int k = 0; k < D; ++k) sx += pdxi[(((int64_t)a * nn + n) * D + j) * D + k] * c[NV + k];
      xbar[pnodes[(int64_t)a * nn + n] * D + j] += sx;
    }
}

template <int D, int P, typename T>
__global__ __launch_bounds__(PROBE_BS) void k_probe_vjp_coef(const T *__restrict__ u, const int64_t *__restrict__ pelem,
                                                             const double *__restrict__ pw,
                                                             const double *__restrict__ pdw, double gm1,
                                                             const double *__restrict__ pbar, bool geo,
                                                             double *__restrict__ coef) {
  constexpr int NC = Shape<D, P>::NV + D;
  probe_vjp_coef_body<D, P, T>(u, pelem, pw, pdw, gm1, pbar, geo, (int)blockIdx.x, coef + (int64_t)blockIdx.x * NC);
}

template <int D, int P, typename T>
__global__ __launch_bounds__(256) void k_probe_vjp_scatter(const int64_t *__restrict__ pelem,
                                                           const double *__restrict__ pw,
                                                           const double *__restrict__ pdxi,
                                                           const int64_t *__restrict__ pnodes, int nn, int n_probe,
                                                           const double *__restrict__ coef, T *ubar, double *xbar) {
  constexpr int NC = Shape<D, P>::NV + D;
  for (int a = 0; a < n_probe; ++a) {
    probe_vjp_scatter_one<D, P, T>(pelem, pw, pdxi, pnodes, nn, a, coef + (int64_t)a * NC, ubar, xbar);
    __syncthreads();  // the next probe may share this element or its nodes
  }
}

template <int D, int P, typename T>
__global__ __launch_bounds__(PROBE_BS) void k_probe_vjp_one(const T *__restrict__ u, const int64_t *__restrict__ pelem,
                                                            const double *__restrict__ pw,
                                                            const double *__restrict__ pdw, double gm1,
                                                            const double *__restrict__ pbar,
                                                            const double *__restrict__ pdxi,
                                                            const int64_t *__restrict__ pnodes, int nn, T *ubar,
                                                            double *xbar) {
  __shared__ double c[Shape<D, P>::NV + D];
  probe_vjp_coef_body<D, P, T>(u, pelem, pw, pdw, gm1, pbar, xbar != nullptr, 0, c);
  __syncthreads();
  probe_vjp_scatter_one<D, P, T>(pelem, pw, pdxi, pnodes, nn, 0, c, ubar, xbar);
}

// RK4 adjoint combination.  init (z == nullptr): a = ub; kb = dt ca ub; zz = 0.
// otherwise: kb = dt (ca a + cz z); ub += z; z = 0 (ready for the next accumulation)
template <typename T>
__global__ void k_rk_adj_combine(T *__restrict__ a, T *__restrict__ z, T *__restrict__ kb, T *__restrict__ ub,
                                 T *__restrict__ zz, double ca, double cz, const double *__restrict__ dt,
                                 const int32_t *__restrict__ elem_mesh, int64_t per_elem, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T d = (T)dt[elem_mesh[i / per_elem]];
  if (!z) {
    const T ai = ub[i];
    a[i] = ai;
    kb[i] = d * (T)ca * ai;
    zz[i] = T(0);
  } else {
    const T zi = z[i];
    kb[i] = d * ((T)ca * a[i] + (T)cz * zi);
    ub[i] += zi;
    z[i] = T(0);
  }
}

template <typename T>
__global__ void k_fill_t(T *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = T(0);
}

// fill kernel (graph-safe replacement for memset)
__global__ void k_fill_f64(double *p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_reset_counters(unsigned long long *count, int *nonfinite) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    count[0] = 0ull;  // sample index
    count[1] = 0ull;  // probe workgroups done in the current sample
    *nonfinite = 0;
  }
}

// ------------------------------------------------------------------------------------ engine
static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// HIP events around one launch when per-kernel timing is enabled (ids FR_K_*)
struct ProfScope {
  const fr_solver *s;
  int id;
  hipStream_t st;
  hipEvent_t a = nullptr;
  static hipEvent_t get(const fr_solver *s) {
    if (!s->prof_pool.empty()) {
      hipEvent_t e = s->prof_pool.back();
      s->prof_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  ProfScope(const fr_solver *s_, int id_, hipStream_t st_) : s(s_), id(id_), st(st_) {
    if (s->profiling) {
      a = get(s);
      (void)hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (s->profiling) {
      hipEvent_t b = get(s);
      (void)hipEventRecord(b, st);
      s->prof_pending.push_back({id, a, b});
    }
  }
};

// launch the candidate tile chosen by the autotuner (index 0: default, 1: half, 2: quarter)
// Autotuner candidates of a volume kernel (kind 0: NS volume, 1: NS lifting + RK, 2: Euler volume
// + RK): index c = (tile size c % 3: the default E, its half, its quarter) x (launch bound c / 3:
// the default and one alternative waves-per-SIMD bound), plus for kind 0 in FP32 3-D p = 4 the
// matrix-core divergence (index 6: default tile, 7: half tile; default bound).  Degree 0 has the
// default only.
template <int V>
using IC = std::integral_constant<int, V>;
template <bool V>
using BC = std::integral_constant<bool, V>;

template <int D, int P, typename T, int KIND>
struct Cands {
  static constexpr int E0 = KIND == 0 ? GradTile<D, P, T>::E : (KIND == 1 ? DivTile<D, P, T>::E : EulerTile<D, P, T>::E);
  using C = TileCands<E0>;
  // waves per SIMD of the alternative bound: the NS volume kernel one wave below its default
  // (more registers per thread), the lifting kernels 8 (at most 64 VGPRs)
  static constexpr int W1 = KIND == 0 ? GradTile<D, P, T>::MIN_WAVES - 1 : 8;
  static constexpr bool HAS_MFMA = KIND == 0 && D == 3 && P == 5 && sizeof(T) == 4;
  static constexpr int N = P == 1 ? 1 : 6 + (HAS_MFMA ? 2 : 0);
  // (elements per workgroup, waves-per-SIMD bound (0: default), engine (1: matrix cores))
  static void list(int32_t *out) {
    const int E[3] = {C::c0, C::c1, C::c2};
    for (int c = 0; c < N; ++c) {
      out[3 * c] = c == 6 ? C::c0 : (c == 7 ? C::c1 : E[c % 3]);
      out[3 * c + 1] = (c >= 3 && c < 6) ? W1 : 0;
      out[3 * c + 2] = c >= 6 ? 1 : 0;
    }
  }
  template <class F>
  static void pick(int c, F &&go) {
    if constexpr (P == 1) {
      go(IC<C::c0>{}, IC<0>{}, BC<false>{});
    } else {
      switch (c) {
        case 1: go(IC<C::c1>{}, IC<0>{}, BC<false>{}); break;
        case 2: go(IC<C::c2>{}, IC<0>{}, BC<false>{}); break;
        case 3: go(IC<C::c0>{}, IC<W1>{}, BC<false>{}); break;
        case 4: go(IC<C::c1>{}, IC<W1>{}, BC<false>{}); break;
        case 5: go(IC<C::c2>{}, IC<W1>{}, BC<false>{}); break;
        case 6:
          if constexpr (HAS_MFMA) {
            go(IC<C::c0>{}, IC<0>{}, BC<true>{});
            break;
          }
          [[fallthrough]];
        case 7:
          if constexpr (HAS_MFMA) {
            go(IC<C::c1>{}, IC<0>{}, BC<true>{});
            break;
          }
          [[fallthrough]];
        default: go(IC<C::c0>{}, IC<0>{}, BC<false>{}); break;
      }
    }
  }
};

template <int D, int P, typename T>
struct Engine {
  using S = Shape<D, P>;

  static OpsDev<T, P> ops(const fr_solver *s) { return make_ops<T, P>(s->ops); }
  static PhysDev<T> phys(const fr_solver *s) {
    PhysDev<T> p;
    p.gamma = (T)s->gamma;
    p.gm1 = (T)(s->gamma - 1.0);
    p.prandtl = (T)s->prandtl;
    p.beta = (T)s->beta;
    p.tau = (T)s->tau;
    p.side = ldg_side_of<T>(s->beta);
    return p;
  }

  static void interp(const fr_solver *s, const T *u, T *uf, hipStream_t st) {
    ProfScope ps(s, 0, st);
    using TL = DivTile<D, P, T>;
    k_interp<D, P, T><<<nblk(s->Ne, TL::E), TL::BS, 0, st>>>(u, uf, s->uf_faces, ops(s), s->Ne);
  }

  // one residual evaluation of `u` whose flux-point values are already in s->uf; the epilogue
  // `rk` decides what is written.  part: bit 0 the volume / common-flux kernels, bit 1 the lifting
  // and RK kernel (a degree group runs the mortar kernels of the whole mesh between the two)
  static void stage(const fr_solver *s, const T *u, const RKArgs<T> &rk, hipStream_t st, bool force_sample,
                    int part = 3) {
    const OpsDev<T, P> o = ops(s);
    const PhysDev<T> ph = phys(s);
    const int64_t nface = s->npair + s->nbnd;
    T *uf = (T *)s->uf, *fhat = (T *)s->fhat;
    const T *metric = (const T *)s->metric;
    const FlowDev<T> *fl = (const FlowDev<T> *)s->flow;
    if (s->equations == 1) {
      T *fvn = (T *)s->fvn, *vol = (T *)s->vol;
      if (part & 1) {
        ProfScope ps(s, 2, st);
        if (s->n_bc < s->nbnd) {  // mortar points: degree-group solver, default tile
          using TL = GradTile<D, P, T, 0>;
          k_ns_grad<D, P, T, 0, true><<<nblk(s->Ne, TL::E), TL::BS, 0, st>>>(
              u, uf, s->nbr, (const T *)s->fnrm, (const T *)s->bnd_nrm, s->n_wall, metric, s->elem_mesh, fl, o,
              ph, fvn, fhat, vol, s->Ne, s->n_bc, (const T *)s->ifc_uh);
        } else {
          auto go = [&](auto te, auto tw, auto tm) {
            constexpr int EE = decltype(te)::value, WW = decltype(tw)::value;
            constexpr bool MF = decltype(tm)::value;
            using TL = GradTile<D, P, T, EE>;
            k_ns_grad<D, P, T, EE, false, WW, MF><<<nblk(s->Ne, TL::E), TL::BS, 0, st>>>(
                u, uf, s->nbr, (const T *)s->fnrm, (const T *)s->bnd_nrm, s->n_wall, metric, s->elem_mesh, fl,
                o, ph, fvn, fhat, vol, s->Ne);
          };
          Cands<D, P, T, 0>::pick(s->tune[0], go);
        }
      }
      if ((part & 1) && force_sample && s->forces && s->n_wall > 0) {
        ProfScope ps(s, 7, st);
        k_wall_force<D, P, T><<<dim3((unsigned)s->wall_nchunk, (unsigned)s->n_mesh), WALL_CHUNK, 0, st>>>(
            uf, fvn, s->bnd, (const T *)s->bnd_nrm, s->bnd_w, s->wall_mesh_begin, ph, s->wall_nchunk,
            s->wall_partial);
        k_wall_force_sum<D><<<s->n_mesh, 64, 0, st>>>(s->wall_partial, s->wall_nchunk, s->force_acc);
      }
      if ((part & 1) && ph.side == 0 && s->npair + s->n_bc > 0) {
        // two-sided LDG (the one-sided common flux is formed in k_ns_grad)
        ProfScope ps(s, 3, st);
        // mortar points (after the first n_bc boundary points) are left to the mortar kernels
        k_face_flux<D, P, T, true><<<nblk(s->npair + s->n_bc, 256), 256, 0, st>>>(
            uf, fvn, s->pairL, s->pairR, (const T *)s->pair_nrm, s->npair, s->bnd, (const T *)s->bnd_nrm,
            s->n_wall, s->n_bc, s->elem_mesh, fl, ph, fhat);
      }
      if (!(part & 2)) return;
      ProfScope ps(s, 4, st);
      auto go = [&](auto te, auto tw, auto) {
        constexpr int EE = decltype(te)::value, WW = decltype(tw)::value;
        using TD = DivTile<D, P, T, EE>;
        if constexpr (WW == 0)
          k_div_rk<D, P, T, EE><<<nblk(s->Ne, TD::E), TD::BS, 0, st>>>(vol, fhat, metric, s->elem_mesh, o, rk, s->Ne);
        else
          k_div_rk_w<D, P, T, EE, WW><<<nblk(s->Ne, TD::E), TD::BS, 0, st>>>(vol, fhat, metric, s->elem_mesh, o, rk,
                                                                             s->Ne);
      };
      Cands<D, P, T, 1>::pick(s->tune[1], go);
    } else {
      {
        ProfScope ps(s, 3, st);
        k_face_flux<D, P, T, false><<<nblk(nface, 256), 256, 0, st>>>(
            uf, nullptr, s->pairL, s->pairR, (const T *)s->pair_nrm, s->npair, s->bnd, (const T *)s->bnd_nrm,
            s->n_wall, s->nbnd, s->elem_mesh, fl, ph, fhat);
      }
      ProfScope ps(s, 5, st);
      auto go = [&](auto te, auto tw, auto) {
        constexpr int EE = decltype(te)::value, WW = decltype(tw)::value;
        using TE = EulerTile<D, P, T, EE>;
        if constexpr (WW == 0)
          k_euler_vol_rk<D, P, T, EE><<<nblk(s->Ne, TE::E), TE::BS, 0, st>>>(u, fhat, metric, s->elem_mesh, o, ph,
                                                                              rk, s->Ne);
        else
          k_euler_vol_rk_w<D, P, T, EE, WW><<<nblk(s->Ne, TE::E), TE::BS, 0, st>>>(u, fhat, metric, s->elem_mesh,
                                                                                   o, ph, rk, s->Ne);
      };
      Cands<D, P, T, 2>::pick(s->tune[2], go);
    }
  }

  static void rhs(const fr_solver *s, const T *u, T *r, hipStream_t st) {
    interp(s, u, (T *)s->uf, st);
    RKArgs<T> rk{};
    rk.r_out = r;
    stage(s, u, rk, st, false);
  }

  // part of the residual of u (flux-point values already in s->uf) into r
  static void rhs_part(const fr_solver *s, const T *u, T *r, int part, hipStream_t st) {
    RKArgs<T> rk{};
    rk.r_out = r;
    stage(s, u, rk, st, false, part);
  }

  // part of stage k of a classical RK4 step of u in place (see step)
  static void stage_k(const fr_solver *s, T *u, const double *dt, int k, bool sample, int part, hipStream_t st) {
    static const double cA[4] = {0.5, 0.5, 1.0, 0.0};
    static const double cB[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    RKArgs<T> rk{};
    rk.u0 = u;
    rk.acc = (T *)s->acc;
    rk.ustage = (T *)s->ustage;
    rk.dt = dt;
    rk.cA = (T)cA[k];
    rk.cB = (T)cB[k];
    rk.first = k == 0;
    rk.last = k == 3;
    rk.uf_next = (T *)s->uf;
    rk.uf_faces = s->uf_faces;
    const T *ust = k == 0 ? u : (const T *)s->ustage;
    stage(s, ust, rk, st, sample && k == 0, part);
  }

  static void probe(const fr_solver *s, const T *u, hipStream_t st) {
    ProfScope ps(s, 6, st);
    if (s->n_probe > 0)
      k_probe<D, P, T><<<(unsigned)s->n_probe, PROBE_BS, 0, st>>>(u, s->probe_elem, s->probe_w, s->probe_pinf,
                                                                   s->gamma - 1.0, s->series, s->cap, s->sums,
                                                                   s->count, s->nonfinite);
    else
      k_probe_count<<<1, 64, 0, st>>>(s->count);
  }

  // one classical RK4 step of u in place; `fresh`: s->uf does not hold u_f of u yet (first step
  // of a call); later steps reuse the flux-point values written by the previous last stage
  static void step(const fr_solver *s, T *u, const double *dt, bool sample, bool fresh, hipStream_t st,
                   T *record = nullptr, T *record_u0 = nullptr, T *record_r = nullptr) {
    static const double cA[4] = {0.5, 0.5, 1.0, 0.0};
    static const double cB[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    if (sample) probe(s, u, st);
    if (fresh) interp(s, u, (T *)s->uf, st);
    for (int k = 0; k < 4; ++k) {
      RKArgs<T> rk{};
      rk.u0 = u;
      rk.acc = (T *)s->acc;
      rk.ustage = (T *)s->ustage;
      rk.dt = dt;
      rk.cA = (T)cA[k];
      rk.cB = (T)cB[k];
      rk.first = k == 0;
      rk.last = k == 3;
      rk.uf_next = (T *)s->uf;
      rk.uf_faces = s->uf_faces;
      rk.ustage_copy = (record && k < 3) ? record + (int64_t)k * s->Ne * S::NV * S::Ns : nullptr;
      rk.u0_copy = k == 0 ? record_u0 : nullptr;
      rk.r_copy = record_r ? record_r + (int64_t)k * s->Ne * S::NV * S::Ns : nullptr;
      const T *ust = k == 0 ? u : (const T *)s->ustage;
      stage(s, ust, rk, st, sample && k == 0);
    }
  }
};

// ------------------------------------------------------------------------------------ dispatch


template <int D, int P, typename T>
Dispatch make_dispatch() {
  Dispatch d;
  d.rhs = [](const fr_solver *s, const void *u, void *r, hipStream_t st) {
    Engine<D, P, T>::rhs(s, (const T *)u, (T *)r, st);
  };
  d.step = [](const fr_solver *s, void *u, const double *dt, bool sample, bool fresh, hipStream_t st) {
    Engine<D, P, T>::step(s, (T *)u, dt, sample, fresh, st);
  };
  d.interp = [](const fr_solver *s, const void *u, hipStream_t st) {
    Engine<D, P, T>::interp(s, (const T *)u, (T *)s->uf, st);
  };
  d.sample_probes = [](const fr_solver *s, const void *u, hipStream_t st) {
    Engine<D, P, T>::probe(s, (const T *)u, st);
  };
  d.rhs_part = [](const fr_solver *s, const void *u, void *r, int part, hipStream_t st) {
    Engine<D, P, T>::rhs_part(s, (const T *)u, (T *)r, part, st);
  };
  d.stage_k = [](const fr_solver *s, void *u, const double *dt, int k, bool sample, int part, hipStream_t st) {
    Engine<D, P, T>::stage_k(s, (T *)u, dt, k, sample, part, st);
  };
  // n steps recording each step's base state (states, optional), its three stage states and
  // (residuals, optional) the residuals of its four stages;
  // flux-point values carry over between the steps of one call, as in fr_rk_step
  d.step_record = [](const fr_solver *s, void *u, const double *dt, int n, void *states, void *stages,
                     void *residuals, hipStream_t st) {
    const int64_t nb = s->Ne * Shape<D, P>::NV * Shape<D, P>::Ns;
    for (int k = 0; k < n; ++k)
      Engine<D, P, T>::step(s, (T *)u, dt, false, k == 0, st, (T *)stages + 3 * nb * k,
                            states ? (T *)states + nb * k : nullptr,
                            residuals ? (T *)residuals + 4 * nb * k : nullptr);
  };
  d.probe_vjp = [](const fr_solver *s, const void *u, const double *pbar, void *ub, double *xbar, hipStream_t st) {
    if (s->n_probe == 1) {
      k_probe_vjp_one<D, P, T><<<1, PROBE_BS, 0, st>>>((const T *)u, s->probe_elem, s->probe_w, s->probe_dw,
                                                       s->gamma - 1.0, pbar, s->probe_dxi, s->probe_nodes,
                                                       s->geo_nn, (T *)ub, xbar);
    } else if (s->n_probe > 1) {
      k_probe_vjp_coef<D, P, T><<<(unsigned)s->n_probe, PROBE_BS, 0, st>>>(
          (const T *)u, s->probe_elem, s->probe_w, s->probe_dw, s->gamma - 1.0, pbar, xbar != nullptr, s->probe_coef);
      k_probe_vjp_scatter<D, P, T><<<1, 256, 0, st>>>(s->probe_elem, s->probe_w, s->probe_dxi, s->probe_nodes,
                                                       s->geo_nn, s->n_probe, s->probe_coef, (T *)ub, xbar);
    }
  };
  d.rk_adj_combine = [](const fr_solver *s, void *a, void *z, void *kb, void *ub, void *zz, double ca, double cz,
                        const double *dt, hipStream_t st) {
    using S = Shape<D, P>;
    const int64_t per = (int64_t)S::NV * S::Ns, n = s->Ne * per;
    k_rk_adj_combine<T><<<nblk(n, 256), 256, 0, st>>>((T *)a, (T *)z, (T *)kb, (T *)ub, (T *)zz, ca, cz, dt,
                                                       s->elem_mesh, per, n);
  };
  d.tune_cands = [](int kind, int32_t *cand) {
    if (kind == 0) {
      Cands<D, P, T, 0>::list(cand);
      return Cands<D, P, T, 0>::N;
    } else if (kind == 1) {
      Cands<D, P, T, 1>::list(cand);
      return Cands<D, P, T, 1>::N;
    }
    Cands<D, P, T, 2>::list(cand);
    return Cands<D, P, T, 2>::N;
  };
  d.zero = [](const fr_solver *s, void *p, hipStream_t st) {
    using S = Shape<D, P>;
    const int64_t n = s->Ne * S::NV * S::Ns;
    k_fill_t<T><<<nblk(n, 256), 256, 0, st>>>((T *)p, n);
  };
  return d;
}

bool get_dispatch(int dim, int p, int precision, Dispatch &out) {
#define FR_CASE(DD, PP)                                                              \
  if (dim == DD && p + 1 == PP) {                                                    \
    out = precision == 0 ? make_dispatch<DD, PP, double>() : make_dispatch<DD, PP, float>(); \
    return true;                                                                     \
  }
  FR_CASE(2, 1) FR_CASE(2, 2) FR_CASE(2, 3) FR_CASE(2, 4) FR_CASE(2, 5)
  FR_CASE(3, 1) FR_CASE(3, 2) FR_CASE(3, 3) FR_CASE(3, 4) FR_CASE(3, 5)
#undef FR_CASE
  return false;
}

void launch_fill(double *p, int64_t n, double v, hipStream_t st) {
  if (n > 0) k_fill_f64<<<nblk(n, 256), 256, 0, st>>>(p, n, v);
}

// zero n values of the state precision
void launch_fill_state(const fr_solver *s, void *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  if (s->precision == 0)
    k_fill_t<double><<<nblk(n, 256), 256, 0, st>>>((double *)p, n);
  else
    k_fill_t<float><<<nblk(n, 256), 256, 0, st>>>((float *)p, n);
}

void launch_reset_counters(unsigned long long *count, int *nonfinite, hipStream_t st) {
  k_reset_counters<<<1, 64, 0, st>>>(count, nonfinite);
}

}  // namespace frmi
