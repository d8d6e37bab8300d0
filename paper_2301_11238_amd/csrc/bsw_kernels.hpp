// HIP kernels of the DG operator, its tangent, the element-block Jacobian and
// the reductions.  One lane per element: the state is stored SoA with the
// element index fastest, so every coefficient load of a wavefront is one
// coalesced 64-element row; the reference tables sit in constant memory and
// are read as wave-uniform scalars.
#pragma once
#include "bsw_device.hpp"

namespace bsw {

extern __constant__ __align__(16) unsigned char c_tables[kTabBytesTotal];

template <int D, int P, class T>
__device__ __forceinline__ const Tab<D, P, T>& tab() {
  return *reinterpret_cast<const Tab<D, P, T>*>(c_tables + tab_offset_rt(D, P, sizeof(T) == 4));
}

// ------------------------------------------------------------------ helpers
template <int D, int P, class T>
__device__ __forceinline__ void load_coeffs(const T* __restrict__ A, int n, int e, T (&c)[Shape<D, P>::NF][Shape<D, P>::NP]) {
#pragma unroll
  for (int f = 0; f < Shape<D, P>::NF; ++f)
#pragma unroll
    for (int i = 0; i < Shape<D, P>::NP; ++i) c[f][i] = A[(size_t)(f * Shape<D, P>::NP + i) * n + e];
}

template <int D, int P, class T>
__device__ __forceinline__ void interp(const T (&phi)[Shape<D, P>::NP], const T (&c)[Shape<D, P>::NF][Shape<D, P>::NP],
                                       T (&X)[Shape<D, P>::NF]) {
#pragma unroll
  for (int f = 0; f < Shape<D, P>::NF; ++f) {
    T s = T(0);
#pragma unroll
    for (int i = 0; i < Shape<D, P>::NP; ++i) s += phi[i] * c[f][i];
    X[f] = s;
  }
}

// neighbour trace: coefficients read from global memory, basis of the
// neighbour's local face g at its point index rr (reversed along the edge)
template <int D, int P, class T>
__device__ __forceinline__ void interp_global(const Tab<D, P, T>& tb, int g, int rr, const T* __restrict__ A, int n,
                                              int nb, T (&X)[Shape<D, P>::NF]) {
#pragma unroll
  for (int f = 0; f < Shape<D, P>::NF; ++f) {
    T s = T(0);
#pragma unroll
    for (int i = 0; i < Shape<D, P>::NP; ++i) s += tb.fphi[g][rr][i] * A[(size_t)(f * Shape<D, P>::NP + i) * n + nb];
    X[f] = s;
  }
}

template <int D, class T>
struct Geo {
  T xi[D][D];  // d xi_r / d x_a
  T detJ;
};

template <int D, class T>
__device__ __forceinline__ void load_geo(const MeshView<T>& m, int e, Geo<D, T>& g) {
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int a = 0; a < D; ++a) g.xi[r][a] = m.dxi[(size_t)(r * D + a) * m.n_el + e];
  g.detJ = m.detJ[e];
}

// Accumulate the test-function contraction at one volume point:
// acc[f][i] += phi_i A[f] + sum_r dphi_ir B[r][f]   for the 1+D balance rows,
// acc[c][i] += phi_i CE[c] + sum_r dphi_ir CB[r][c] for the D*D gradient rows.
template <int D, int P, class T>
__device__ __forceinline__ void contract_volume(const Tab<D, P, T>& tb, int q, const T (&A)[1 + D], const T (&B)[D][1 + D],
                                                const T (&CE)[D * D], const T (&CB)[D][D * D],
                                                T (&acc)[Shape<D, P>::NF][Shape<D, P>::NP]) {
  using S = Shape<D, P>;
#pragma unroll
  for (int i = 0; i < S::NP; ++i) {
    const T ph = tb.phi[q][i];
#pragma unroll
    for (int f = 0; f <= D; ++f) {
      T v = ph * A[f];
#pragma unroll
      for (int r = 0; r < D; ++r) v += tb.dphi[q][i][r] * B[r][f];
      acc[f][i] += v;
    }
#pragma unroll
    for (int c = 0; c < D * D; ++c) {
      T v = ph * CE[c];
#pragma unroll
      for (int r = 0; r < D; ++r) v += tb.dphi[q][i][r] * CB[r][c];
      acc[1 + D + c][i] += v;
    }
  }
}

// Pointwise volume integrand of Eq. WeakForm7 at one point (weight wq):
// balance rows: A = wq (U/dt - S), B[r] = -wq sum_a xi_ra (F_a - Q_a);
// gradient rows (c = b*D + a): CE = wq E_ab, CB[r] = wq xi_ra u_b.
template <int D, class T>
__device__ __forceinline__ void volume_integrand(const DevParams<T>& p, const Geo<D, T>& g, T wq, const Pt<D, T>& s,
                                                 const Stress<D, T>& st, T (&A)[1 + D], T (&B)[D][1 + D],
                                                 T (&CE)[D * D], T (&CB)[D][D * D]) {
  T G[D][1 + D];  // F_a - Q_a
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const T hua = s.h * s.u[a];
    G[a][0] = hua;
#pragma unroll
    for (int b = 0; b < D; ++b)
      G[a][1 + b] = hua * s.u[b] + (a == b ? T(0.5) * p.gc * s.h * s.h : T(0)) - s.h * st.sig[b][a] * p.rho_inv;
  }
  A[0] = wq * s.h * p.inv_dt;
#pragma unroll
  for (int b = 0; b < D; ++b) A[1 + b] = wq * (s.h * s.u[b] * p.inv_dt + (b == 0 ? p.gs * s.h : T(0)));
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int f = 0; f <= D; ++f) {
      T v = T(0);
#pragma unroll
      for (int a = 0; a < D; ++a) v += g.xi[r][a] * G[a][f];
      B[r][f] = -wq * v;
    }
#pragma unroll
  for (int b = 0; b < D; ++b)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      CE[b * D + a] = wq * s.E[a][b];
#pragma unroll
      for (int r = 0; r < D; ++r) CB[r][b * D + a] = wq * g.xi[r][a] * s.u[b];
    }
}

// Its directional derivative (Appendix A: dU/dV, dF/dV, dQ/dV, dQ/dE, dS/dV,
// dG/dV); the gradient rows are linear.
template <int D, class T>
__device__ __forceinline__ void volume_integrand_tan(const DevParams<T>& p, const Geo<D, T>& g, T wq,
                                                     const Pt<D, T>& s, const Stress<D, T>& st, const Pt<D, T>& ds,
                                                     T (&A)[1 + D], T (&B)[D][1 + D], T (&CE)[D * D],
                                                     T (&CB)[D][D * D]) {
  T dsig[D][D];
  stress_tan<D, T>(st, ds.E, dsig);
  T G[D][1 + D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const T hua = s.h * s.u[a];
    const T dhua = ds.h * s.u[a] + s.h * ds.u[a];
    G[a][0] = dhua;
#pragma unroll
    for (int b = 0; b < D; ++b)
      G[a][1 + b] = dhua * s.u[b] + hua * ds.u[b] + (a == b ? p.gc * s.h * ds.h : T(0)) -
                    (ds.h * st.sig[b][a] + s.h * dsig[b][a]) * p.rho_inv;
  }
  A[0] = wq * ds.h * p.inv_dt;
#pragma unroll
  for (int b = 0; b < D; ++b)
    A[1 + b] = wq * ((ds.h * s.u[b] + s.h * ds.u[b]) * p.inv_dt + (b == 0 ? p.gs * ds.h : T(0)));
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int f = 0; f <= D; ++f) {
      T v = T(0);
#pragma unroll
      for (int a = 0; a < D; ++a) v += g.xi[r][a] * G[a][f];
      B[r][f] = -wq * v;
    }
#pragma unroll
  for (int b = 0; b < D; ++b)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      CE[b * D + a] = wq * ds.E[a][b];
#pragma unroll
      for (int r = 0; r < D; ++r) CB[r][b * D + a] = wq * g.xi[r][a] * ds.u[b];
    }
}

// Face integrand: balance rows get w (F_hll.n - Q_central.n), gradient rows
// get -w u_central,b n_a (Sec. 5, Eqs. HLLSolver and the central fluxes).
template <int D, class T>
__device__ __forceinline__ void face_flux(const DevParams<T>& p, const T* n, T wr, const Pt<D, T>& sm, const Pt<D, T>& sp,
                                          T (&FV)[1 + D], T (&FE)[D * D]) {
  HLLState<D, T> H;
  T Fn[1 + D];
  hll<D, T>(p, sm, sp, n, H, Fn);
  Stress<D, T> qm, qp;
  stress<D, T>(p, sm.E, qm);
  stress<D, T>(p, sp.E, qp);
  FV[0] = wr * Fn[0];
#pragma unroll
  for (int b = 0; b < D; ++b) {
    T qn = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) qn += (sm.h * qm.sig[b][a] + sp.h * qp.sig[b][a]) * n[a];
    FV[1 + b] = wr * (Fn[1 + b] - T(0.5) * qn * p.rho_inv);
  }
#pragma unroll
  for (int b = 0; b < D; ++b)
#pragma unroll
    for (int a = 0; a < D; ++a) FE[b * D + a] = -wr * T(0.5) * (sm.u[b] + sp.u[b]) * n[a];
}

template <int D, class T>
__device__ __forceinline__ void face_flux_tan(const DevParams<T>& p, const T* n, T wr, const Pt<D, T>& sm,
                                              const Pt<D, T>& sp, const Pt<D, T>& dsm, const Pt<D, T>& dsp,
                                              T (&FV)[1 + D], T (&FE)[D * D]) {
  HLLState<D, T> H;
  T Fn[1 + D], dFn[1 + D];
  hll<D, T>(p, sm, sp, n, H, Fn);
  hll_tan<D, T>(p, H, sm, sp, dsm, dsp, n, dFn);
  Stress<D, T> qm, qp;
  stress<D, T>(p, sm.E, qm);
  stress<D, T>(p, sp.E, qp);
  T dsm_sig[D][D], dsp_sig[D][D];
  stress_tan<D, T>(qm, dsm.E, dsm_sig);
  stress_tan<D, T>(qp, dsp.E, dsp_sig);
  FV[0] = wr * dFn[0];
#pragma unroll
  for (int b = 0; b < D; ++b) {
    T qn = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a)
      qn += (dsm.h * qm.sig[b][a] + sm.h * dsm_sig[b][a] + dsp.h * qp.sig[b][a] + sp.h * dsp_sig[b][a]) * n[a];
    FV[1 + b] = wr * (dFn[1 + b] - T(0.5) * qn * p.rho_inv);
  }
#pragma unroll
  for (int b = 0; b < D; ++b)
#pragma unroll
    for (int a = 0; a < D; ++a) FE[b * D + a] = -wr * T(0.5) * (dsm.u[b] + dsp.u[b]) * n[a];
}

template <int D, int P, class T>
__device__ __forceinline__ void lift_face(const Tab<D, P, T>& tb, int fc, int rr, const T (&FV)[1 + D], const T (&FE)[D * D],
                                          T (&acc)[Shape<D, P>::NF][Shape<D, P>::NP]) {
#pragma unroll
  for (int i = 0; i < Shape<D, P>::NP; ++i) {
    const T ph = tb.fphi[fc][rr][i];
#pragma unroll
    for (int f = 0; f <= D; ++f) acc[f][i] += ph * FV[f];
#pragma unroll
    for (int c = 0; c < D * D; ++c) acc[1 + D + c][i] += ph * FE[c];
  }
}

// ------------------------------------------------------------------ kernels
// b_old = (1/dt) <phi, U(W_old)> on the 1+D balance rows.
template <int D, int P, class T>
__global__ void __launch_bounds__(256) k_step_begin(const T* __restrict__ W, T* __restrict__ bold, MeshView<T> m,
                                                     DevParams<T> p) {
  using S = Shape<D, P>;
  const Tab<D, P, T>& tb = tab<D, P, T>();
  const int n = m.n_el;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  T w[S::NF][S::NP];
  load_coeffs<D, P, T>(W, n, e, w);
  T acc[S::NV][S::NP];
#pragma unroll
  for (int f = 0; f < S::NV; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) acc[f][i] = T(0);
  const T detJ = m.detJ[e];
#pragma unroll
  for (int q = 0; q < S::NQ; ++q) {
    T X[S::NF];
    interp<D, P, T>(tb.phi[q], w, X);
    const T c = tb.qw[q] * detJ * p.inv_dt;
    T U[S::NV];
    U[0] = c * X[0];
#pragma unroll
    for (int b = 0; b < D; ++b) U[1 + b] = c * X[0] * X[1 + b];
#pragma unroll
    for (int i = 0; i < S::NP; ++i)
#pragma unroll
      for (int f = 0; f < S::NV; ++f) acc[f][i] += tb.phi[q][i] * U[f];
  }
#pragma unroll
  for (int f = 0; f < S::NV; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) bold[(size_t)(f * S::NP + i) * n + e] = acc[f][i];
}

// R = residual of Eq. WeakForm7 (element-centric; each element evaluates the
// numerical fluxes on its own faces from its own and its neighbour's traces).
template <int D, int P, class T>
__global__ void __launch_bounds__(256) k_operator(const T* __restrict__ W, const T* __restrict__ bold,
                                                   T* __restrict__ R, MeshView<T> m, DevParams<T> p) {
  using S = Shape<D, P>;
  const Tab<D, P, T>& tb = tab<D, P, T>();
  const int n = m.n_el;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  T w[S::NF][S::NP];
  load_coeffs<D, P, T>(W, n, e, w);
  Geo<D, T> g;
  load_geo<D, T>(m, e, g);
  T acc[S::NF][S::NP];
#pragma unroll
  for (int f = 0; f < S::NF; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) acc[f][i] = T(0);
#pragma unroll 1
  for (int q = 0; q < S::NQ; ++q) {
    T X[S::NF];
    interp<D, P, T>(tb.phi[q], w, X);
    Pt<D, T> s;
    unpack<D, T>(X, s);
    Stress<D, T> st;
    stress<D, T>(p, s.E, st);
    T A[1 + D], B[D][1 + D], CE[D * D], CB[D][D * D];
    volume_integrand<D, T>(p, g, tb.qw[q] * g.detJ, s, st, A, B, CE, CB);
    contract_volume<D, P, T>(tb, q, A, B, CE, CB, acc);
  }
#pragma unroll
  for (int f = 0; f < S::NV; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) acc[f][i] -= bold[(size_t)(f * S::NP + i) * n + e];
#pragma unroll 1
  for (int fc = 0; fc < S::NFC; ++fc) {
    const int code = m.nbr[(size_t)fc * n + e];
    T nv[D];
#pragma unroll
    for (int a = 0; a < D; ++a) nv[a] = m.nrm[(size_t)(fc * D + a) * n + e];
    const T hl = m.hlen[(size_t)fc * n + e];
#pragma unroll 1
    for (int rr = 0; rr < S::NFQ; ++rr) {
      T Xm[S::NF];
      interp<D, P, T>(tb.fphi[fc][rr], w, Xm);
      Pt<D, T> sm, sp;
      unpack<D, T>(Xm, sm);
      if (code >= 0) {
        T Xp[S::NF];
        interp_global<D, P, T>(tb, code & 3, S::NFQ - 1 - rr, W, n, code >> 2, Xp);
        unpack<D, T>(Xp, sp);
      } else {
        exterior<D, T>(p, nv, sm, sp);
      }
      T FV[1 + D], FE[D * D];
      face_flux<D, T>(p, nv, tb.fw[rr] * hl, sm, sp, FV, FE);
      lift_face<D, P, T>(tb, fc, rr, FV, FE, acc);
    }
  }
#pragma unroll
  for (int f = 0; f < S::NF; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) R[(size_t)(f * S::NP + i) * n + e] = acc[f][i];
}

// Tangent of the element residual.  The perturbation is either a full vector
// x (matrix-free Jacobian product: own and neighbour coefficients) or the
// unit vector of one own degree of freedom (a column of the diagonal block).
template <int D, int P, class T, bool COLUMN>
__device__ __forceinline__ void elem_tangent(const Tab<D, P, T>& tb, const T* __restrict__ W, const T* __restrict__ x,
                                             const MeshView<T>& m, const DevParams<T>& p, int e, int col,
                                             T (&acc)[Shape<D, P>::NF][Shape<D, P>::NP]) {
  using S = Shape<D, P>;
  const int n = m.n_el;
  T w[S::NF][S::NP];
  load_coeffs<D, P, T>(W, n, e, w);
  T v[COLUMN ? 1 : S::NF][COLUMN ? 1 : S::NP];
  if constexpr (!COLUMN) load_coeffs<D, P, T>(x, n, e, v);
  const int cf = COLUMN ? col / S::NP : 0;
  const int ci = COLUMN ? col % S::NP : 0;
  Geo<D, T> g;
  load_geo<D, T>(m, e, g);
#pragma unroll
  for (int f = 0; f < S::NF; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) acc[f][i] = T(0);
#pragma unroll 1
  for (int q = 0; q < S::NQ; ++q) {
    T X[S::NF], dX[S::NF];
    interp<D, P, T>(tb.phi[q], w, X);
    if constexpr (COLUMN) {
#pragma unroll
      for (int f = 0; f < S::NF; ++f) dX[f] = (f == cf) ? tb.phi[q][ci] : T(0);
    } else {
      interp<D, P, T>(tb.phi[q], v, dX);
    }
    Pt<D, T> s, ds;
    unpack<D, T>(X, s);
    unpack<D, T>(dX, ds);
    Stress<D, T> st;
    stress<D, T>(p, s.E, st);
    T A[1 + D], B[D][1 + D], CE[D * D], CB[D][D * D];
    volume_integrand_tan<D, T>(p, g, tb.qw[q] * g.detJ, s, st, ds, A, B, CE, CB);
    contract_volume<D, P, T>(tb, q, A, B, CE, CB, acc);
  }
#pragma unroll 1
  for (int fc = 0; fc < S::NFC; ++fc) {
    const int code = m.nbr[(size_t)fc * n + e];
    T nv[D];
#pragma unroll
    for (int a = 0; a < D; ++a) nv[a] = m.nrm[(size_t)(fc * D + a) * n + e];
    const T hl = m.hlen[(size_t)fc * n + e];
#pragma unroll 1
    for (int rr = 0; rr < S::NFQ; ++rr) {
      T Xm[S::NF], dXm[S::NF];
      interp<D, P, T>(tb.fphi[fc][rr], w, Xm);
      if constexpr (COLUMN) {
#pragma unroll
        for (int f = 0; f < S::NF; ++f) dXm[f] = (f == cf) ? tb.fphi[fc][rr][ci] : T(0);
      } else {
        interp<D, P, T>(tb.fphi[fc][rr], v, dXm);
      }
      Pt<D, T> sm, sp, dsm, dsp;
      unpack<D, T>(Xm, sm);
      unpack<D, T>(dXm, dsm);
      if (code >= 0) {
        T Xp[S::NF];
        interp_global<D, P, T>(tb, code & 3, S::NFQ - 1 - rr, W, n, code >> 2, Xp);
        unpack<D, T>(Xp, sp);
        if constexpr (COLUMN) {
          T z[S::NF];
#pragma unroll
          for (int f = 0; f < S::NF; ++f) z[f] = T(0);
          unpack<D, T>(z, dsp);
        } else {
          T dXp[S::NF];
          interp_global<D, P, T>(tb, code & 3, S::NFQ - 1 - rr, x, n, code >> 2, dXp);
          unpack<D, T>(dXp, dsp);
        }
      } else {
        exterior<D, T>(p, nv, sm, sp);
        exterior_tan<D, T>(p, nv, dsm, dsp);
      }
      T FV[1 + D], FE[D * D];
      face_flux_tan<D, T>(p, nv, tb.fw[rr] * hl, sm, sp, dsm, dsp, FV, FE);
      lift_face<D, P, T>(tb, fc, rr, FV, FE, acc);
    }
  }
}

template <int D, int P, class T>
__global__ void __launch_bounds__(256) k_jac_apply(const T* __restrict__ W, const T* __restrict__ x, T* __restrict__ y,
                                                    MeshView<T> m, DevParams<T> p) {
  using S = Shape<D, P>;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.n_el) return;
  T acc[S::NF][S::NP];
  elem_tangent<D, P, T, false>(tab<D, P, T>(), W, x, m, p, e, 0, acc);
#pragma unroll
  for (int f = 0; f < S::NF; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) y[(size_t)(f * S::NP + i) * m.n_el + e] = acc[f][i];
}

// Column `col` of every diagonal block: blocks[(row * BS + col) * n_el + e].
template <int D, int P, class T>
__global__ void __launch_bounds__(256) k_jac_columns(const T* __restrict__ W, T* __restrict__ blocks, MeshView<T> m,
                                                      DevParams<T> p) {
  using S = Shape<D, P>;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int col = blockIdx.y;
  if (e >= m.n_el) return;
  T acc[S::NF][S::NP];
  elem_tangent<D, P, T, true>(tab<D, P, T>(), W, nullptr, m, p, e, col, acc);
#pragma unroll
  for (int f = 0; f < S::NF; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) blocks[((size_t)(f * S::NP + i) * S::BS + col) * m.n_el + e] = acc[f][i];
}

// In-place LU with partial pivoting of every block ([BS][BS][n_el] layout);
// perm[k][e] = original row of factor row k.  One lane per element.
template <int BS, class T>
__global__ void __launch_bounds__(256) k_block_lu(T* __restrict__ A, int* __restrict__ perm, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  auto a = [&](int r, int c) -> T& { return A[((size_t)r * BS + c) * n + e]; };
  for (int k = 0; k < BS; ++k) perm[(size_t)k * n + e] = k;
  for (int k = 0; k < BS; ++k) {
    int pv = k;
    T big = fabs(a(k, k));
    for (int r = k + 1; r < BS; ++r) {
      const T v = fabs(a(r, k));
      if (v > big) { big = v; pv = r; }
    }
    if (pv != k) {
      for (int c = 0; c < BS; ++c) { const T t = a(k, c); a(k, c) = a(pv, c); a(pv, c) = t; }
      const int t = perm[(size_t)k * n + e];
      perm[(size_t)k * n + e] = perm[(size_t)pv * n + e];
      perm[(size_t)pv * n + e] = t;
    }
    const T inv = T(1) / a(k, k);
    for (int r = k + 1; r < BS; ++r) {
      const T l = a(r, k) * inv;
      a(r, k) = l;
      for (int c = k + 1; c < BS; ++c) a(r, c) -= l * a(k, c);
    }
  }
}

// y = U^{-1} L^{-1} P x per element (x and y in the state layout).
template <int BS, class T>
__global__ void __launch_bounds__(256) k_block_solve(const T* __restrict__ LU, const int* __restrict__ perm,
                                                      const T* __restrict__ x, T* __restrict__ y, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  T v[BS];
#pragma unroll
  for (int k = 0; k < BS; ++k) v[k] = x[(size_t)perm[(size_t)k * n + e] * n + e];
#pragma unroll
  for (int i = 1; i < BS; ++i) {
    T s = v[i];
#pragma unroll
    for (int j = 0; j < i; ++j) s -= LU[((size_t)i * BS + j) * n + e] * v[j];
    v[i] = s;
  }
#pragma unroll
  for (int i = BS - 1; i >= 0; --i) {
    T s = v[i];
#pragma unroll
    for (int j = i + 1; j < BS; ++j) s -= LU[((size_t)i * BS + j) * n + e] * v[j];
    v[i] = s / LU[((size_t)i * BS + i) * n + e];
  }
#pragma unroll
  for (int k = 0; k < BS; ++k) y[(size_t)k * n + e] = v[k];
}

}  // namespace bsw
