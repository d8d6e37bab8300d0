// HIP kernels of the DG operator, its tangent, the element-block Jacobian and
// the reductions.  The state is stored SoA with the element index fastest, so
// the coefficient loads of consecutive elements coalesce.  The reference
// tables sit in constant memory; where the lanes of a wave read different
// entries (different points or modes) those reads take the vector memory path.
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
// Face traces: the values of every field at every face point of an element,
// tr[(f * NFP + kp) * n + e] with kp = face * NFQ + point.  One coalesced pass
// per state; an element then reads its neighbour's side of a shared face
// point as NF loads instead of interpolating NF x NP neighbour coefficients.
// one item: field f on face fc of element e, item = (f * NFC + fc) * n + e
template <int D, int P, class T>
__device__ __forceinline__ void trace_item(const T* __restrict__ X, T* __restrict__ tr, int n, int64_t item) {
  using S = Shape<D, P>;
  const Tab<D, P, T>& tb = tab<D, P, T>();
  constexpr int NFP = S::NFC * S::NFQ;
  const int e = (int)(item % n);
  const int ff = (int)(item / n);
  const int f = ff / S::NFC, fc = ff % S::NFC;
  T c[S::NP];
#pragma unroll
  for (int i = 0; i < S::NP; ++i) c[i] = X[(size_t)(f * S::NP + i) * n + e];
#pragma unroll
  for (int r = 0; r < S::NFQ; ++r) {
    T s = T(0);
#pragma unroll
    for (int i = 0; i < S::NP; ++i) s += tb.fphi[fc][r][i] * c[i];
    tr[(size_t)(f * NFP + fc * S::NFQ + r) * n + e] = s;
  }
}

template <int D, int P, class T>
__global__ void __launch_bounds__(256) k_trace(const T* __restrict__ X, T* __restrict__ tr, int n) {
  const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (item < (int64_t)Shape<D, P>::NF * Shape<D, P>::NFC * n) trace_item<D, P, T>(X, tr, n, item);
}

// the neighbour's values at its local face g, point rr (points run in the
// opposite direction along a shared edge)
template <int D, int P, class T>
__device__ __forceinline__ void load_trace(const T* __restrict__ tr, int n, int nb, int g, int rr,
                                           T (&X)[Shape<D, P>::NF]) {
  using S = Shape<D, P>;
  constexpr int NFP = S::NFC * S::NFQ;
  const int kp = g * S::NFQ + rr;
#pragma unroll
  for (int f = 0; f < S::NF; ++f) X[f] = tr[(size_t)(f * NFP + kp) * n + nb];
}

// The field values at face point rr of face g of element nb, from its
// coefficients X (the values trace_item stores, in the same arithmetic):
// the Jacobian apply evaluates the neighbour's side of x this way instead of
// reading a trace array written by a separate pass.
template <int D, int P, class T>
__device__ __forceinline__ void neighbour_values(const Tab<D, P, T>& tb, const T* __restrict__ X, int n, int nb,
                                                 int g, int rr, T (&V)[Shape<D, P>::NF]) {
  using S = Shape<D, P>;
#pragma unroll
  for (int f = 0; f < S::NF; ++f) {
    T c[S::NP];
#pragma unroll
    for (int i = 0; i < S::NP; ++i) c[i] = X[(size_t)(f * S::NP + i) * n + nb];
    T s = T(0);
#pragma unroll
    for (int i = 0; i < S::NP; ++i) s += tb.fphi[g][rr][i] * c[i];
    V[f] = s;
  }
}

// Mixed orders (Sec. 5: m1, m2, m3 for h, u and E).  The bases are ordered by
// total degree, so field f of order m lives in the span of its first N(m)
// modes and is tested with them; the rows of the higher modes carry the
// trivial equations W = 0 (residual row = coefficient, identity Jacobian row).
// The diagonal blocks also drop those modes' columns, so the preconditioner
// keeps them exactly zero.
// (One packed word: choosing among three loaded fields by a runtime field
// index would make the compiler address the descriptor in scratch memory.)
template <int D, class T>
__device__ __forceinline__ bool row_unused(const MeshView<T>& m, int f, int i) {
  const int sel = f == 0 ? 0 : (f <= D ? 8 : 16);
  return i >= ((m.nmodes >> sel) & 255);
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

// Momentum source of Eq. Sterm per unit depth at volume point q: S_b = -sl_b h
// with sl_b = g_s [b = 0] + g_c dH/dx_b.  The bed gradient comes from the
// element's bed coefficients and the affine metric.
template <int D, int P, class T>
__device__ __forceinline__ void source_slope(const Tab<D, P, T>& tb, int q, const Geo<D, T>& g, const MeshView<T>& m,
                                             const DevParams<T>& p, int e, T (&sl)[D]) {
  sl[0] = p.gs;
#pragma unroll
  for (int b = 1; b < D; ++b) sl[b] = T(0);
  if (m.bed) {
    T dr[D];
#pragma unroll
    for (int r = 0; r < D; ++r) dr[r] = T(0);
#pragma unroll
    for (int i = 0; i < Shape<D, P>::NP; ++i) {
      const T Hi = m.bed[(size_t)i * m.n_el + e];
#pragma unroll
      for (int r = 0; r < D; ++r) dr[r] += tb.dphi[q][i][r] * Hi;
    }
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T v = T(0);
#pragma unroll
      for (int r = 0; r < D; ++r) v += g.xi[r][b] * dr[r];
      sl[b] += p.gc * v;
    }
  }
}

// Pointwise volume integrand of Eq. WeakForm7 at one point (weight wq):
// balance rows: A = wq (U/dt - S), B[r] = -wq sum_a xi_ra (F_a - Q_a);
// gradient rows (c = b*D + a): CE = wq E_ab, CB[r] = wq xi_ra u_b.
// sl is the source slope of the point (source_slope).
template <int D, class T>
__device__ __forceinline__ void volume_integrand(const DevParams<T>& p, const Geo<D, T>& g, T wq, const Pt<D, T>& s,
                                                 const Stress<D, T>& st, const T (&sl)[D], T (&A)[1 + D],
                                                 T (&B)[D][1 + D], T (&CE)[D * D], T (&CB)[D][D * D]) {
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
  for (int b = 0; b < D; ++b) A[1 + b] = wq * (s.h * s.u[b] * p.inv_dt + sl[b] * s.h);
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
                                                     const T (&sl)[D], T (&A)[1 + D], T (&B)[D][1 + D],
                                                     T (&CE)[D * D], T (&CB)[D][D * D]) {
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
    A[1 + b] = wq * ((ds.h * s.u[b] + s.h * ds.u[b]) * p.inv_dt + sl[b] * ds.h);
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
__device__ __forceinline__ void step_begin_elem(const T* __restrict__ W, T* __restrict__ bold, const MeshView<T>& m,
                                                const DevParams<T>& p, int e) {
  using S = Shape<D, P>;
  const Tab<D, P, T>& tb = tab<D, P, T>();
  const int n = m.n_el;
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

template <int D, int P, class T>
__global__ void __launch_bounds__(256) k_step_begin(const T* __restrict__ W, T* __restrict__ bold, MeshView<T> m,
                                                     DevParams<T> p) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m.n_el) step_begin_elem<D, P, T>(W, bold, m, p, e);
}

// Workgroups are dealt round-robin to the chip's 8 XCDs, each with its own L2.
// Map hardware workgroup b to element tile t so that every XCD gets one
// contiguous run of tiles: face neighbours (adjacent elements and the
// neighbouring row of a structured mesh) then mostly hit the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  constexpr int kXcd = 8;
  const int q = nb / kXcd, r = nb % kXcd;
  const int x = b % kXcd, k = b / kXcd;
  return x * q + (x < r ? x : r) + k;
}

// ------------------------------------------------------------------ blocked kernels
// A workgroup takes EB consecutive elements.  Their coefficients are staged in
// LDS with one coalesced pass; then one lane per (element, quadrature point)
// and per (element, face point) evaluates the pointwise integrand and parks it
// in LDS; then one lane per (element, output row) contracts it with the test
// functions and writes the row.  This keeps every lane's live state to one
// point (no register spills at P3 in FP64) and gives NQ + NFC*NFQ lanes per
// element instead of one.  NT is the workgroup size (the element-tile shape:
// EB = NT / (NQ + NFC*NFQ) elements); every NT gives the same bits, the
// autotuner picks the fastest per order, precision and size class.
constexpr int kTileShapes = 3;
constexpr int kTileNT[kTileShapes] = {128, 256, 512};

// Waves per SIMD the element pass is compiled for (register budget 512 / w):
// 3 for the FP64 order-3 triangle (its point lanes need about 165 registers),
// 4 otherwise.
template <int D, int P, class T>
constexpr int elem_waves() { return (D == 2 && P == 3 && sizeof(T) == 8) ? 3 : 4; }

template <int D, int P, int NT = 256>
struct Blk {
  using S = Shape<D, P>;
  static constexpr int NFP = S::NFC * S::NFQ;                          // face points per element
  static constexpr int NPT = S::NQ + NFP;                              // point items per element
  static constexpr int EB = NT / NPT;                                  // elements per workgroup
  static constexpr int OA = 0;                                         // A[f]
  static constexpr int OB = 1 + D;                                     // B[r][f]
  static constexpr int OCE = OB + D * (1 + D);                         // CE[c]
  static constexpr int OCB = OCE + D * D;                              // CB[r][c]
  static constexpr int NVF = OCB + D * D * D;                          // reals per volume point
  static constexpr int NFF = 1 + D + D * D;                            // reals per face point
};

// MODE 0: residual (x unused, bold subtracted; trW unused: the neighbours'
// side of W is evaluated here); MODE 1: Jacobian product along x (bold
// unused; the neighbours' side of W from the linearisation's traces trW, that
// of x evaluated here).  One tile: elements e0 .. e0+EB-1 of one mesh.
template <int D, int P, class T, int MODE, int NT = 256>
__device__ __forceinline__ void elem_blocked_tile(const T* __restrict__ W, const T* __restrict__ x,
                                                  const T* __restrict__ bold, T* __restrict__ out,
                                                  const T* __restrict__ trW, const MeshView<T>& m,
                                                  const DevParams<T>& p, int e0) {
  using S = Shape<D, P>;
  using B = Blk<D, P, NT>;
  constexpr bool TAN = MODE == 1;
  const Tab<D, P, T>& tb = tab<D, P, T>();
  const int n = m.n_el;
  const int tid = threadIdx.x;
  __shared__ T sW[S::BS][B::EB];
  __shared__ T sX[TAN ? S::BS : 1][TAN ? B::EB : 1];
  __shared__ T sV[S::NQ][B::NVF][B::EB];
  __shared__ T sF[B::NFP][B::NFF][B::EB];

  for (int idx = tid; idx < S::BS * B::EB; idx += NT) {
    const int row = idx / B::EB, el = idx % B::EB, e = e0 + el;
    sW[row][el] = e < n ? W[(size_t)row * n + e] : T(0);
    if constexpr (TAN) sX[row][el] = e < n ? x[(size_t)row * n + e] : T(0);
  }
  __syncthreads();

  if (tid < B::EB * B::NPT) {
    const int el = tid % B::EB, k = tid / B::EB, e = e0 + el;
    if (e < n) {
      if (k < S::NQ) {
        const int q = k;
        Geo<D, T> g;
        load_geo<D, T>(m, e, g);
        T X[S::NF];
#pragma unroll
        for (int f = 0; f < S::NF; ++f) {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < S::NP; ++i) s += tb.phi[q][i] * sW[f * S::NP + i][el];
          X[f] = s;
        }
        Pt<D, T> s;
        unpack<D, T>(X, s);
        Stress<D, T> st;
        stress<D, T>(p, s.E, st);
        T A[1 + D], Bm[D][1 + D], CE[D * D], CB[D][D * D];
        const T wq = tb.qw[q] * g.detJ;
        T sl[D];
        source_slope<D, P, T>(tb, q, g, m, p, e, sl);
        if constexpr (TAN) {
          T dX[S::NF];
#pragma unroll
          for (int f = 0; f < S::NF; ++f) {
            T s2 = T(0);
#pragma unroll
            for (int i = 0; i < S::NP; ++i) s2 += tb.phi[q][i] * sX[f * S::NP + i][el];
            dX[f] = s2;
          }
          Pt<D, T> ds;
          unpack<D, T>(dX, ds);
          volume_integrand_tan<D, T>(p, g, wq, s, st, ds, sl, A, Bm, CE, CB);
        } else {
          volume_integrand<D, T>(p, g, wq, s, st, sl, A, Bm, CE, CB);
        }
#pragma unroll
        for (int f = 0; f <= D; ++f) sV[q][B::OA + f][el] = A[f];
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
          for (int f = 0; f <= D; ++f) sV[q][B::OB + r * (1 + D) + f][el] = Bm[r][f];
#pragma unroll
        for (int c = 0; c < D * D; ++c) sV[q][B::OCE + c][el] = CE[c];
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
          for (int c = 0; c < D * D; ++c) sV[q][B::OCB + r * D * D + c][el] = CB[r][c];
      } else {
        const int kp = k - S::NQ, fc = kp / S::NFQ, rr = kp % S::NFQ;
        const int code = m.nbr[(size_t)fc * n + e];
        T nv[D];
#pragma unroll
        for (int a = 0; a < D; ++a) nv[a] = m.nrm[(size_t)(fc * D + a) * n + e];
        const T wr = tb.fw[rr] * m.hlen[(size_t)fc * n + e];
        T Xm[S::NF], dXm[S::NF];
#pragma unroll
        for (int f = 0; f < S::NF; ++f) {
          T s1 = T(0), s2 = T(0);
#pragma unroll
          for (int i = 0; i < S::NP; ++i) {
            s1 += tb.fphi[fc][rr][i] * sW[f * S::NP + i][el];
            if constexpr (TAN) s2 += tb.fphi[fc][rr][i] * sX[f * S::NP + i][el];
          }
          Xm[f] = s1;
          dXm[f] = s2;
        }
        Pt<D, T> sm, sp, dsm, dsp;
        unpack<D, T>(Xm, sm);
        if constexpr (TAN) unpack<D, T>(dXm, dsm);
        if (code >= 0) {
          T Xp[S::NF];
          // residual: the neighbour's side of W evaluated here; Jacobian:
          // from the linearisation's traces of W
          if constexpr (TAN) load_trace<D, P, T>(trW, n, code >> 2, code & 3, S::NFQ - 1 - rr, Xp);
          else neighbour_values<D, P, T>(tb, W, n, code >> 2, code & 3, S::NFQ - 1 - rr, Xp);
          unpack<D, T>(Xp, sp);
          if constexpr (TAN) {
            T dXp[S::NF];
            neighbour_values<D, P, T>(tb, x, n, code >> 2, code & 3, S::NFQ - 1 - rr, dXp);
            unpack<D, T>(dXp, dsp);
          }
        } else {
          exterior<D, T>(p, nv, -1 - code, sm, sp);
          if constexpr (TAN) exterior_tan<D, T>(p, nv, -1 - code, dsm, dsp);
        }
        T FV[1 + D], FE[D * D];
        if constexpr (TAN) face_flux_tan<D, T>(p, nv, wr, sm, sp, dsm, dsp, FV, FE);
        else face_flux<D, T>(p, nv, wr, sm, sp, FV, FE);
#pragma unroll
        for (int f = 0; f <= D; ++f) sF[kp][f][el] = FV[f];
#pragma unroll
        for (int c = 0; c < D * D; ++c) sF[kp][1 + D + c][el] = FE[c];
      }
    }
  }
  __syncthreads();

  for (int idx = tid; idx < S::BS * B::EB; idx += NT) {
    const int row = idx / B::EB, el = idx % B::EB, e = e0 + el;
    if (e >= n) continue;
    const int f = row / S::NP, i = row % S::NP;
    if (row_unused<D, T>(m, f, i)) {
      T v;
      if constexpr (TAN) v = sX[row][el];
      else v = sW[row][el];
      out[(size_t)row * n + e] = v;
      continue;
    }
    T acc = T(0);
    if (f <= D) {
#pragma unroll
      for (int q = 0; q < S::NQ; ++q) {
        acc += tb.phi[q][i] * sV[q][B::OA + f][el];
#pragma unroll
        for (int r = 0; r < D; ++r) acc += tb.dphi[q][i][r] * sV[q][B::OB + r * (1 + D) + f][el];
      }
#pragma unroll
      for (int kp = 0; kp < B::NFP; ++kp) acc += tb.fphi[kp / S::NFQ][kp % S::NFQ][i] * sF[kp][f][el];
      if constexpr (!TAN) acc -= bold[(size_t)row * n + e];
    } else {
      const int c = f - (1 + D);
#pragma unroll
      for (int q = 0; q < S::NQ; ++q) {
        acc += tb.phi[q][i] * sV[q][B::OCE + c][el];
#pragma unroll
        for (int r = 0; r < D; ++r) acc += tb.dphi[q][i][r] * sV[q][B::OCB + r * D * D + c][el];
      }
#pragma unroll
      for (int kp = 0; kp < B::NFP; ++kp) acc += tb.fphi[kp / S::NFQ][kp % S::NFQ][i] * sF[kp][1 + D + c][el];
    }
    out[(size_t)row * n + e] = acc;
  }
}

template <int D, int P, class T, int MODE>
__global__ void __launch_bounds__(256, (elem_waves<D, P, T>())) k_elem_blocked(const T* __restrict__ W, const T* __restrict__ x,
                                                       const T* __restrict__ bold, T* __restrict__ out,
                                                       const T* __restrict__ trW, MeshView<T> m, DevParams<T> p) {
  elem_blocked_tile<D, P, T, MODE>(W, x, bold, out, trW, m, p,
                                   xcd_tile(blockIdx.x, gridDim.x) * Blk<D, P>::EB);
}

// Tangent of the element residual along the unit vector of one own degree of
// freedom, col = f * N_p + i (a column of the diagonal block): the neighbour's
// side is held fixed.  wl: the element's coefficients (row f * N_p + i), in
// LDS and shared by the lanes of the element's columns.
template <int D, int P, class T>
__device__ __forceinline__ void column_tangent(const Tab<D, P, T>& tb, const T* wl, const T* __restrict__ trW,
                                               const MeshView<T>& m, const DevParams<T>& p, int e, int col,
                                               T (&acc)[Shape<D, P>::NF][Shape<D, P>::NP]) {
  using S = Shape<D, P>;
  const int n = m.n_el;
  auto at = [&](const T (&phi)[S::NP], T (&X)[S::NF]) {
#pragma unroll
    for (int f = 0; f < S::NF; ++f) {
      T s = T(0);
#pragma unroll
      for (int i = 0; i < S::NP; ++i) s += phi[i] * wl[f * S::NP + i];
      X[f] = s;
    }
  };
  const int cf = col / S::NP;
  const int ci = col % S::NP;
  Geo<D, T> g;
  load_geo<D, T>(m, e, g);
#pragma unroll
  for (int f = 0; f < S::NF; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) acc[f][i] = T(0);
#pragma unroll 1
  for (int q = 0; q < S::NQ; ++q) {
    T X[S::NF], dX[S::NF];
    at(tb.phi[q], X);
#pragma unroll
    for (int f = 0; f < S::NF; ++f) dX[f] = (f == cf) ? tb.phi[q][ci] : T(0);
    Pt<D, T> s, ds;
    unpack<D, T>(X, s);
    unpack<D, T>(dX, ds);
    Stress<D, T> st;
    stress<D, T>(p, s.E, st);
    T A[1 + D], B[D][1 + D], CE[D * D], CB[D][D * D];
    T sl[D];
    source_slope<D, P, T>(tb, q, g, m, p, e, sl);
    volume_integrand_tan<D, T>(p, g, tb.qw[q] * g.detJ, s, st, ds, sl, A, B, CE, CB);
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
      at(tb.fphi[fc][rr], Xm);
#pragma unroll
      for (int f = 0; f < S::NF; ++f) dXm[f] = (f == cf) ? tb.fphi[fc][rr][ci] : T(0);
      Pt<D, T> sm, sp, dsm, dsp;
      unpack<D, T>(Xm, sm);
      unpack<D, T>(dXm, dsm);
      if (code >= 0) {
        T Xp[S::NF];
        load_trace<D, P, T>(trW, n, code >> 2, code & 3, S::NFQ - 1 - rr, Xp);
        unpack<D, T>(Xp, sp);
        T z[S::NF];
#pragma unroll
        for (int f = 0; f < S::NF; ++f) z[f] = T(0);
        unpack<D, T>(z, dsp);
      } else {
        exterior<D, T>(p, nv, -1 - code, sm, sp);
        exterior_tan<D, T>(p, nv, -1 - code, dsm, dsp);
      }
      T FV[1 + D], FE[D * D];
      face_flux_tan<D, T>(p, nv, tb.fw[rr] * hl, sm, sp, dsm, dsp, FV, FE);
      lift_face<D, P, T>(tb, fc, rr, FV, FE, acc);
    }
  }
}

// Diagonal-block columns: one lane per column, the lanes of a 256-thread
// workgroup packed with the columns of as many whole elements as fit (six at
// BS = 42, three at BS = 70), so that few lanes idle.
template <int BS>
constexpr int cols_epb() { return 256 / BS; }
constexpr int cols_tiles_for(int bs, int n) { return (n + 256 / bs - 1) / (256 / bs); }

template <int D, int P, class T>
__device__ __forceinline__ void jac_columns_elem(const T* __restrict__ W, const T* __restrict__ trW,
                                                 T* __restrict__ blocks, const MeshView<T>& m, const DevParams<T>& p,
                                                 int g) {
  using S = Shape<D, P>;
  constexpr int EPB = cols_epb<S::BS>();
  const int col = threadIdx.x % S::BS, el = (int)threadIdx.x / S::BS, e = g * EPB + el;
  const bool live = (int)threadIdx.x < EPB * S::BS && e < m.n_el;
  // the element's coefficients, once per element in LDS (lane col loads entry col)
  __shared__ T wl[EPB][S::BS];
  if (live) wl[el][col] = W[(size_t)col * m.n_el + e];
  __syncthreads();
  if (!live) return;
  T acc[S::NF][S::NP];
  column_tangent<D, P, T>(tab<D, P, T>(), wl[el], trW, m, p, e, col, acc);
  T* blk = blocks + (size_t)e * S::BS * S::BS;
#pragma unroll
  for (int f = 0; f < S::NF; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) {
      const int row = f * S::NP + i;
      const bool trivial = row_unused<D, T>(m, f, i) || row_unused<D, T>(m, col / S::NP, col % S::NP);
      blk[row * S::BS + col] = trivial ? T(row == col ? 1 : 0) : acc[f][i];
    }
}

template <int D, int P, class T>
__global__ void __launch_bounds__(256) k_jac_columns(const T* __restrict__ W, const T* __restrict__ trW,
                                                      T* __restrict__ blocks, MeshView<T> m, DevParams<T> p) {
  jac_columns_elem<D, P, T>(W, trW, blocks, m, p, blockIdx.x);
}

// Inverse of one diagonal block per workgroup: Gauss-Jordan elimination with
// partial pivoting on [A | I], in place.  Each lane keeps one row in
// registers.  Rows are never swapped: the lane whose row supplies the pivot of
// step k (largest |entry| in the current column among the rows not yet used,
// lowest row on ties) supplies it to the other lanes, which subtract its
// multiple: by lane reads into scalar registers when the block fits one wave,
// through LDS (one barrier per step) when it spans two.  The register row is rotated by one position per step, so the
// current column is always register 0 and the step body is the same for every
// step (a loop, not BS unrolled copies): position j takes the updated entry of
// position j + 1, and the last position takes the new column of the right-hand
// part.  Pivot rows are not normalised when chosen; each lane divides its row
// by its own pivot at the end, which commutes with the later eliminations.
// After BS steps the lane that supplied pivot k holds row k of the inverse,
// its position k' the column piv[k'].
// The inverse is written element-fastest, Ainv[(row * BS + col) * n + e], so
// the preconditioner apply is a coalesced batched mat-vec.  It is stored in
// FP32 for both state precisions: the preconditioner only steers GMRES (the
// Krylov residual uses the exact Jacobian), and its apply reads half the bytes.
// Consecutive elements run on one XCD, so the elements that share a line of
// the output fill it in the same L2.
template <int BS>
constexpr int inv_threads() { return 64 * ((BS + 63) / 64); }
// waves per SIMD the inversion is compiled for (FP64 rows of 70 fit 3)
template <int BS, class T>
constexpr int inv_waves() { return BS > 64 && sizeof(T) == 8 ? 3 : 4; }

// the device library's wave reduction of 64-bit keys (its 32-bit siblings are
// declared by the HIP headers)
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_max_u64(unsigned long long);

// integer keys of non-negative floats (their bit patterns order like the values)
template <class T> struct PivotKey;
// (wave_max: the maximum over all 64 lanes of the wave, every lane active)
template <> struct PivotKey<double> {
  using U = unsigned long long;
  static __device__ __forceinline__ U bits(double v) { return (U)__double_as_longlong(v); }
  static __device__ __forceinline__ double value(U k) { return __longlong_as_double((long long)k); }
  static __device__ __forceinline__ U wave_max(U k) { return __ockl_wfred_max_u64(k); }
};
template <> struct PivotKey<float> {
  using U = unsigned int;
  static __device__ __forceinline__ U bits(float v) { return (U)__float_as_uint(v); }
  static __device__ __forceinline__ float value(U k) { return __uint_as_float(k); }
  static __device__ __forceinline__ U wave_max(U k) { return __ockl_wfred_max_u32(k); }
};

// the value v holds in lane l of the wave (l wave-uniform), as a scalar
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int BS, class T>
__device__ __forceinline__ void block_inverse_elem(const T* __restrict__ A, float* __restrict__ Ainv, int n, int e) {
  constexpr int NT = inv_threads<BS>();
  constexpr int NW = NT / 64;
  // per-wave pivot candidates (value, row, the row itself), double-buffered
  // by step parity so that one barrier per step suffices
  __shared__ T crow[2][NW][BS];
  __shared__ T cval[2][NW];
  __shared__ int cidx[2][NW];
  __shared__ int piv[BS];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const bool own = t < BS;
  const T* src = A + (size_t)e * BS * BS + (size_t)(own ? t : 0) * BS;
  T r[BS];
#pragma unroll
  for (int j = 0; j < BS; ++j) r[j] = own ? src[j] : T(0);
  bool used = !own;
  int myk = 0;
  T dp = T(1);  // the lane's own pivot value
  for (int k = 0; k < BS; ++k) {
    const int buf = k & 1;
    // the wave's pivot candidate: largest |entry| among its rows not yet used,
    // lowest row on ties, as two wave reductions on an integer key (the bits
    // of a non-negative float order like its value; used rows key 0).  A NaN
    // entry counts as the largest, so the pivot is always a row not yet used
    // (every row is used exactly once and piv[] stays a permutation).
    T av = fabs(r[0]);
    if (av != av) av = T(INFINITY);
    using K = typename PivotKey<T>::U;
    const K key = used ? K(0) : PivotKey<T>::bits(av) + K(1);
    const K mx = PivotKey<T>::wave_max(key);
    int bi = (int)__ockl_wfred_min_u32(key == mx ? (unsigned)t : 0xffffffffu);
    T best = mx == K(0) ? T(-1) : PivotKey<T>::value(mx - K(1));
    if constexpr (NW == 1) {
      // one wave: the pivot row is read from the pivot lane's registers into
      // scalar registers (no LDS traffic and no barrier per step)
      bi = __builtin_amdgcn_readfirstlane(bi);
      const bool me = t == bi;
      const T d = lane_value(r[0], bi);
      if (me) { used = true; myk = k; dp = d; }
      if (t == 0) piv[k] = bi;
      const T f = me ? T(0) : r[0] / d;
#pragma unroll
      for (int j = 0; j + 1 < BS; ++j) r[j] = r[j + 1] - f * lane_value(r[j + 1], bi);
      r[BS - 1] = me ? T(1) : -f;
    } else {
      if (t == bi) {
#pragma unroll
        for (int j = 0; j < BS; ++j) crow[buf][wv][j] = r[j];
      }
      if (lane == 0) { cval[buf][wv] = best; cidx[buf][wv] = bi; }
      __syncthreads();
      int w = 0;
      best = cval[buf][0];
      bi = cidx[buf][0];
#pragma unroll
      for (int u = 1; u < NW; ++u)
        if (cval[buf][u] > best || (cval[buf][u] == best && cidx[buf][u] < bi)) { best = cval[buf][u]; bi = cidx[buf][u]; w = u; }
      const T* prow = crow[buf][w];
      const bool me = t == bi;
      if (me) { used = true; myk = k; dp = prow[0]; }
      if (t == 0) piv[k] = bi;
      const T f = me ? T(0) : r[0] / prow[0];
#pragma unroll
      for (int j = 0; j + 1 < BS; ++j) r[j] = r[j + 1] - f * prow[j + 1];
      r[BS - 1] = me ? T(1) : -f;
    }
  }
  __syncthreads();
  if (own) {
    const T s = T(1) / dp;
    float* dst = Ainv + (size_t)myk * BS * n + e;
#pragma unroll
    for (int j = 0; j < BS; ++j) dst[(size_t)piv[j] * n] = (float)(r[j] * s);
  }
}

template <int BS, class T>
__global__ void __launch_bounds__(inv_threads<BS>(), (inv_waves<BS, T>())) k_block_inverse(const T* __restrict__ A, float* __restrict__ Ainv,
                                                                     int n) {
  block_inverse_elem<BS, T>(A, Ainv, n, xcd_tile(blockIdx.x, gridDim.x));
}

// y = blockdiag(A_e)^{-1} x: one lane per (row, element), element fastest.
// A launch tile is 256 elements of one row, and consecutive tiles take the
// rows of the same elements (tile t: row t % BS, elements (t / BS) * 256 +
// lane), so the BS rows of an element tile reuse its slice of x from the L2
// of one XCD instead of refetching it from HBM for every row.
template <int BS>
__device__ __forceinline__ void row_tile(int t, int& row, int& e) {
  row = t % BS;
  e = (t / BS) * 256 + (int)threadIdx.x;
}

template <int BS, class T>
__device__ __forceinline__ void block_apply_item(const float* __restrict__ Ainv, const T* __restrict__ x,
                                                 T* __restrict__ y, int n, int row, int e) {
  const float* arow = Ainv + (size_t)row * BS * n + e;
  T s = T(0);
#pragma unroll
  for (int j = 0; j < BS; ++j) s += (T)arow[(size_t)j * n] * x[(size_t)j * n + e];
  y[(size_t)row * n + e] = s;
}

template <int BS, class T>
__global__ void __launch_bounds__(256) k_block_apply(const float* __restrict__ Ainv, const T* __restrict__ x,
                                                      T* __restrict__ y, int n) {
  int row, e;
  row_tile<BS>(xcd_tile(blockIdx.x, gridDim.x), row, e);
  if (e < n) block_apply_item<BS, T>(Ainv, x, y, n, row, e);
}

// per-element contributions to the mass, the active (yielded) area, the
// largest |u| + sqrt(g h) and the smallest depth over the volume points
template <int D, int P, class T>
__device__ __forceinline__ void diag_elem(const T* __restrict__ W, const MeshView<T>& m, double g, double thr, int e,
                                          double (&v)[4]) {
  using S = Shape<D, P>;
  const Tab<D, P, T>& tb = tab<D, P, T>();
  const int n = m.n_el;
  {
    T w[S::NF][S::NP];
    load_coeffs<D, P, T>(W, n, e, w);
    const double detJ = (double)m.detJ[e];
#pragma unroll
    for (int q = 0; q < S::NQ; ++q) {
      T X[S::NF];
      interp<D, P, T>(tb.phi[q], w, X);
      const double wq = (double)tb.qw[q] * detJ;
      const double h = (double)X[0];
      v[0] += wq * h;
      double tr = 0.0, n2 = 0.0, um = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) tr += (double)X[1 + D + a * D + a];
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
          const double dab = 0.5 * ((double)X[1 + D + b * D + a] + (double)X[1 + D + a * D + b]);
          n2 += dab * dab;
        }
      const double s = sqrt(0.5 * (n2 + tr * tr));
      if (s - thr >= 0.0) v[1] += wq;
#pragma unroll
      for (int b = 0; b < D; ++b) um += (double)X[1 + b] * (double)X[1 + b];
      v[2] = fmax(v[2], sqrt(um) + sqrt(g * fmax(h, 0.0)));
      v[3] = fmin(v[3], h);
    }
  }
}

}  // namespace bsw
