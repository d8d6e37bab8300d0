// HIP kernels of the DG operator, its tangent, the element-block Jacobian and
// the reductions.  The state is stored SoA with the element index fastest, so
// the coefficient loads of consecutive elements coalesce.  The reference
// tables sit in constant memory and are read through the scalar unit at
// wave-uniform indices; where the lanes of a wave read different entries the
// block assembly stages the tables in LDS, and the element pass reads its one
// such table (the neighbour's face basis) through the vector memory path.
#pragma once
#include "bsw_device.hpp"

namespace bsw {

extern __constant__ __align__(16) unsigned char c_tables[kTabBytesTotal];

// Entry e of row `row` of an element-fastest array with n columns.  The row
// base is wave-uniform (scalar registers) and the byte offset of e is formed
// in 32 bits (a row block of one call stays below 4 GiB), so a load needs
// little address arithmetic per lane.
template <class T>
__device__ __forceinline__ T rowld(const T* __restrict__ a, int row, int n, unsigned e) {
  const char* r = reinterpret_cast<const char*>(a + (size_t)row * (size_t)n);
  return *reinterpret_cast<const T*>(r + e * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ T& rowref(T* a, int row, int n, unsigned e) {
  char* r = reinterpret_cast<char*>(a + (size_t)row * (size_t)n);
  return *reinterpret_cast<T*>(r + e * (unsigned)sizeof(T));
}

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

// ---------------------------------------------------------------- block-Jacobi
// The preconditioner is the inverse of the block diagonal of the Jacobian,
// applied through the Schur complement of each block's stress part.  The
// rows of a block split into the depth and velocity rows V (fields h, u;
// NV = (1 + D) N_p, the velocity rows U = N_p .. NV - 1) and the stress rows E
// (D^2 N_p).  The discrete equations fix three zero or diagonal parts:
//  * the stress equations (Sec. 3, the mixed form of the velocity gradient)
//    are algebraic and linear in E with the element mass matrix, which is
//    |J| I for the orthonormal basis: A_EE = D is diagonal;
//  * the depth equation does not involve E, and the stress equations do not
//    involve h: A_hE = 0 and A_Eh = 0.
// So the Schur complement S = A_VV - A_VE D^{-1} A_EV differs from A_VV only
// in its U x U part, and the block solve z = A^{-1} x is
//   z_V = S^{-1} (x_V - A_VE D^{-1} x_E),   z_E = D^{-1} x_E - D^{-1} A_EU z_U.
// Per element the factors S^{-1} (NV x NV) and G = A_UE (NU x NE) are stored,
// in FP32 and element fastest (number k of element e at F[k * n + e]).  On
// triangles D^{-1} A_EU and D^{-1} are not stored: the stress equations'
// dependence on the velocity is linear with state-independent coefficients
// (the weak gradient: the volume term and the central face trace), so
// D^{-1} A_EU z_U is evaluated in the apply from the element's geometry, its
// boundary codes and the reference tables, and D = |J| I; 1700 numbers per
// element at P3 against 4900 for the whole inverse, from a 30-row inversion
// instead of a 70-row one.  In 1-D H = D^{-1} A_EU (NE x NU) and d = D^{-1}
// (NE) are stored too.  FP32 for both state precisions: the preconditioner
// only steers GMRES (the Krylov residual uses the exact Jacobian) and its
// apply reads half the bytes.  A_EE's off-diagonal entries are quadrature
// rounding of zero (about 1e-13 of the diagonal) and are not read.
template <int D, int P>
struct Schur {
  static constexpr int NP = Shape<D, P>::NP;
  static constexpr int BS = Shape<D, P>::BS;
  static constexpr int NV = (1 + D) * NP;  // depth and velocity rows
  static constexpr int NU = D * NP;        // velocity rows, NP .. NV - 1
  static constexpr int NE = D * D * NP;    // stress rows, NV .. BS - 1
  static constexpr bool GEO = D == 2;     // D^{-1} A_EU from the geometry
  static constexpr int OS = 0;             // S^{-1}, row-major
  static constexpr int OG = NV * NV;       // G = A_UE, row-major
  static constexpr int OH = OG + NU * NE;  // H = D^{-1} A_EU, row-major (1-D)
  static constexpr int OD = OH + NE * NU;  // d = D^{-1} (1-D)
  static constexpr int NB = GEO ? OH : OD + NE;  // numbers per element
  // the factor build's inputs: on triangles the compact parts the
  // linearisation assembles (per element A_VV row-major, A_UE row-major,
  // A_EU row-major, diag A_EE; CB numbers), in 1-D whole row-major blocks
  static constexpr int CUE = NV * NV, CEU = CUE + NU * NE, CDG = CEU + NE * NU;
  static constexpr int CB = GEO ? CDG + NE : BS * BS;
  static_assert(NV <= 64, "the Schur complement rows must fit one wave");
};
// numbers per element of the stored factors (host side)
constexpr int schur_numbers(int dim, int np) {
  return ((1 + dim) * np) * ((1 + dim) * np) + (dim == 2 ? 1 : 2) * (dim * np) * (dim * dim * np) +
         (dim == 2 ? 0 : dim * dim * np);
}

// the device library's wave reduction of 64-bit keys (its 32-bit siblings are
// declared by the HIP headers)
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_max_u64(unsigned long long);

// integer keys of non-negative floats (their bit patterns order like the values)
template <class T> struct PivotKey;
// (wave_max: the maximum over all 64 lanes of the wave, every lane active)
template <> struct PivotKey<double> {
  using U = unsigned long long;
  static __device__ __forceinline__ U bits(double v) { return (U)__double_as_longlong(v); }
  static __device__ __forceinline__ U wave_max(U k) { return __ockl_wfred_max_u64(k); }
};
template <> struct PivotKey<float> {
  using U = unsigned int;
  static __device__ __forceinline__ U bits(float v) { return (U)__float_as_uint(v); }
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

// The factors of element e from its diagonal block A (the compact factor
// inputs of Schur on triangles, [e][number]; whole row-major blocks in 1-D)
// by one wave of a four-wave workgroup (every wave reaches the barrier; live
// is false for a wave past the last element, whose loads then read element
// 0's block and whose results are dropped).  D^{-1}, A_EU and the velocity
// lanes' A_UE entries go to the wave's slice of LDS (in 1-D D^{-1} A_EU and
// D^{-1} are also stored as factors).  Lane t < NV holds row t of S in
// registers: the row of A_VV, minus (velocity rows) the products of its A_UE
// entries, scaled by D^{-1}, with the rows of A_EU, read back from LDS as
// broadcasts one stress row at a time.  The loads of each phase go out
// together, before their first use.  S is inverted by Gauss-Jordan
// elimination with partial pivoting on [S | I], in place and without row
// swaps: at step k the lane whose row has the largest |entry| in the current
// column among the rows not yet used (lowest row on ties) supplies the pivot
// row, which the other lanes read from its registers lane by lane.  The
// register row is rotated by one position per step, so the current column is
// always position 0 and every step runs the same code: position j takes the
// updated entry of position j + 1 and the last position the new column of the
// right-hand part.  Pivot rows are not normalised when chosen; each lane
// divides its row by its own pivot at the end, which commutes with the later
// eliminations.  After NV steps the lane that supplied pivot k holds row k of
// S^{-1}, its position j the column of the row that supplied pivot j.
constexpr int kSchurEPB = 4;  // elements (waves) per workgroup
template <int D, int P, class T>
__device__ __forceinline__ void schur_build_elem(const T* __restrict__ A, float* __restrict__ F, int n, int e,
                                                 bool live) {
  using Z = Schur<D, P>;
  constexpr int NH = Z::NE * Z::NU;
  constexpr int JH = (NH + 63) / 64;  // entries of D^{-1} A_EU per lane
  constexpr int KC = Z::NE % 20 == 0 ? 20 : (Z::NE % 8 == 0 ? 8 : Z::NE);  // A_UE entries per batch
  __shared__ T sD[kSchurEPB][Z::NE];
  __shared__ T sA[kSchurEPB][Z::NE][Z::NU];  // A_EU
  __shared__ T sG[kSchurEPB][Z::NE][Z::NU];  // A_UE, transposed (velocity lane fastest)
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const T* blk = A + (size_t)(live ? e : 0) * Z::CB;
  float* out = F + (live ? e : 0);
  const bool own = live && lane < Z::NV;
  const bool vel = own && lane >= Z::NP;
  // the lane's row of A_VV and, for a velocity lane, of A_UE
  const int rl = lane < Z::NV ? lane : 0;
  const T* row = blk + (size_t)rl * (Z::GEO ? Z::NV : Z::BS);
  const T* urow = Z::GEO ? blk + Z::CUE + (size_t)(rl >= Z::NP ? rl - Z::NP : 0) * Z::NE : row + Z::NV;
  T a[JH];
#pragma unroll
  for (int j = 0; j < JH; ++j) {
    const int i = lane + 64 * j < NH ? lane + 64 * j : 0;
    a[j] = Z::GEO ? blk[Z::CEU + i] : blk[(size_t)(Z::NV + i / Z::NU) * Z::BS + Z::NP + i % Z::NU];
  }
  const int kd = lane < Z::NE ? lane : 0;
  const T dd = Z::GEO ? blk[Z::CDG + kd] : blk[(size_t)(Z::NV + kd) * Z::BS + Z::NV + kd];
  T r[Z::NV];
#pragma unroll
  for (int c = 0; c < Z::NV; ++c) r[c] = row[c];
  if (lane < Z::NE) {
    const T di = T(1) / dd;
    sD[w][lane] = di;
    if (!Z::GEO && live) out[(size_t)(Z::OD + lane) * n] = (float)di;
  }
  __syncthreads();
  if constexpr (!Z::GEO) {
#pragma unroll
    for (int j = 0; j < JH; ++j) {
      const int i = lane + 64 * j;
      if (live && i < NH) out[(size_t)(Z::OH + i) * n] = (float)(a[j] * sD[w][i / Z::NU]);
    }
  }
  // A_EU (raw) and the velocity lanes' A_UE entries to the wave's LDS slice;
  // the A_UE entries also go out as the factor G
  float* gout = out + (size_t)(Z::OG + (vel ? lane - Z::NP : 0) * Z::NE) * n;
#pragma unroll
  for (int j = 0; j < JH; ++j) {
    const int i = lane + 64 * j;
    if (i < NH) sA[w][i / Z::NU][i % Z::NU] = a[j];
  }
#pragma unroll 1
  for (int k0 = 0; k0 < Z::NE; k0 += KC) {
    T g[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) g[kk] = urow[k0 + kk];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      if (vel) {
        gout[(size_t)(k0 + kk) * n] = (float)g[kk];
        sG[w][k0 + kk][lane - Z::NP] = g[kk];
      }
    }
  }
  __syncthreads();
  // S_UU -= A_UE D^{-1} A_EU, one stress row k at a time: the lane's A_UE
  // entry and row k of A_EU (a broadcast) from LDS
#pragma unroll 2
  for (int k = 0; k < Z::NE; ++k) {
    const T f = vel ? sG[w][k][lane - Z::NP] * sD[w][k] : T(0);
#pragma unroll
    for (int c = 0; c < Z::NU; ++c) r[Z::NP + c] -= f * sA[w][k][c];
  }
  if (!live) return;
  bool used = !own;
  int myk = 0, pv = 0;
  T dp = T(1);  // the lane's own pivot value
  for (int k = 0; k < Z::NV; ++k) {
    // pivot: largest |entry| among the rows not yet used, lowest row on ties,
    // as two wave reductions on an integer key (used rows key 0).  A NaN entry
    // counts as the largest, so every row is used exactly once.
    T av = fabs(r[0]);
    if (av != av) av = T(INFINITY);
    using K = typename PivotKey<T>::U;
    const K key = used ? K(0) : PivotKey<T>::bits(av) + K(1);
    const K mx = PivotKey<T>::wave_max(key);
    const int bi = __builtin_amdgcn_readfirstlane((int)__ockl_wfred_min_u32(key == mx ? (unsigned)lane : 0xffffffffu));
    const bool me = lane == bi;
    const T dv = lane_value(r[0], bi);
    if (me) { used = true; myk = k; dp = dv; }
    if (lane == k) pv = bi;
    const T f = me ? T(0) : r[0] / dv;
#pragma unroll
    for (int j = 0; j + 1 < Z::NV; ++j) r[j] = r[j + 1] - f * lane_value(r[j + 1], bi);
    r[Z::NV - 1] = me ? T(1) : -f;
  }
  if (own) {
    const T s = T(1) / dp;
    float* srow = out + (size_t)(Z::OS + myk * Z::NV) * n;
#pragma unroll
    for (int j = 0; j < Z::NV; ++j) srow[(size_t)__builtin_amdgcn_readlane(pv, j) * n] = (float)(r[j] * s);
  }
}

// consecutive elements run on one XCD, so the elements that share a line of
// the output fill it in one L2
template <int D, int P, class T>
__global__ void __launch_bounds__(256) k_schur_build(const T* __restrict__ A, float* __restrict__ F, int n) {
  const int e = xcd_tile(blockIdx.x, gridDim.x) * kSchurEPB + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  schur_build_elem<D, P, T>(A, F, n, e, e < n);
}

// On triangles, row (b, a, k) of D^{-1} A_EU z_U (stress row E_ab, mode k;
// z_U the velocity coefficients), from the element's residual of the weak
// gradient: the volume term sum_q w_q |J| (grad phi_k . xi_.a) u_b and the
// face term -sum_r w_r (|face| / 2) phi_k (u_b^- + u_b^+) / 2 n_a, whose
// own-side derivative carries I + du^+/du^- with du^+/du^- = 0 across interior faces
// and at Dirichlet faces, I at Neumann faces and I - 2 n n^T at walls (the
// exterior states of the boundary kinds); divided by D = |J|.  zq: z_b at the
// volume points; zf[fc][rr][c]: z_c at the face points (unused velocity
// modes masked out: their columns of A_EU are unit columns of the block).
// emit(k, hz_k) receives row k; the loop over k is kept rolled so that only
// one mode's reference-table entries are live (unrolled, the compiler hoists
// all of them into scalar registers and spills those).
template <int P, class T, class Emit>
__device__ __forceinline__ void schur_geo_rows(const Tab<2, P, T>& tb, const MeshView<T>& m, int bc, unsigned e,
                                               int b, int a, const double (&zq)[Shape<2, P>::NQ],
                                               const double (&zf)[3][Shape<2, P>::NFQ][2], Emit emit) {
  using S = Shape<2, P>;
  const int n = m.n_el;
  const double inv_det = 1.0 / (double)rowld(m.detJ, 0, n, e);
  const double xa0 = (double)rowld(m.dxi, 0 * 2 + a, n, e), xa1 = (double)rowld(m.dxi, 1 * 2 + a, n, e);
  // the face coefficients c_fc[rr] = sum_c beta_fc[b][c] zf[fc][rr][c], with
  // the factor -(|face| / 2) n_a / (2 |J|) (hlen holds |face| / 2)
  double cf[3][S::NFQ];
#pragma unroll
  for (int fc = 0; fc < 3; ++fc) {
    const int code = rowld(m.nbr, fc, n, e);
    const double n0 = (double)rowld(m.nrm, fc * 2 + 0, n, e), n1 = (double)rowld(m.nrm, fc * 2 + 1, n, e);
    const double hl = (double)rowld(m.hlen, fc, n, e);
    int kind = 0;  // 0: the exterior side is fixed (interior face or Dirichlet)
    if (code < 0) {
      const int cb = -1 - code;
      kind = (cb & 3) ? (cb & 3) : bc;
      if (kind == 3) kind = 0;
    }
    const double nb = b == 0 ? n0 : n1, na = a == 0 ? n0 : n1;
    // beta row b
    double b0 = b == 0 ? 1.0 : 0.0, b1 = b == 1 ? 1.0 : 0.0;
    if (kind == 2) { b0 *= 2.0; b1 *= 2.0; }
    if (kind == 1) { b0 = 2.0 * (b0 - nb * n0); b1 = 2.0 * (b1 - nb * n1); }
    const double sc = -0.5 * hl * na * inv_det;
#pragma unroll
    for (int rr = 0; rr < S::NFQ; ++rr) cf[fc][rr] = sc * (double)tb.fw[rr] * (b0 * zf[fc][rr][0] + b1 * zf[fc][rr][1]);
  }
#pragma unroll 1
  for (int k = 0; k < S::NP; ++k) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < S::NQ; ++q)
      v += (double)tb.qw[q] * ((double)tb.dphi[q][k][0] * xa0 + (double)tb.dphi[q][k][1] * xa1) * zq[q];
#pragma unroll
    for (int fc = 0; fc < 3; ++fc)
#pragma unroll
      for (int rr = 0; rr < S::NFQ; ++rr) v += (double)tb.fphi[fc][rr][k] * cf[fc][rr];
    emit(k, v);
  }
}

// Block solve of 64 consecutive elements by a workgroup of four waves, one
// lane per element.  x is staged in LDS (the stress rows already scaled by
// D^{-1}); then r_U = x_U - G t_E replaces x_U, z_V = S^{-1} r_V is written
// and z_U replaces r_U, and z_E = t_E - D^{-1} A_EU z_U is written (on
// triangles each wave takes one stress field and forms D^{-1} A_EU z_U from
// the geometry; in 1-D from the stored H).  The waves take the rows of each
// phase in turn.  Every factor row is a coalesced read of 64 consecutive FP32
// numbers.  scale() (called once by every thread, after the first phase)
// gives the factor applied to the written z.  m and bc (the boundary kind of
// faces coded 0) serve the geometric rows.
constexpr int kPrecEB = 64;
template <int D, int P, class T, class Scale>
__device__ __forceinline__ void schur_apply_tile(const float* __restrict__ F, const T* __restrict__ x,
                                                 T* __restrict__ y, const MeshView<T>& m, int bc, int e0,
                                                 Scale scale) {
  using Z = Schur<D, P>;
  using S = Shape<D, P>;
  constexpr int NW = 4;
  const int n = m.n_el;
  __shared__ double xs[Z::BS][kPrecEB];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const unsigned e = (unsigned)(e0 + lane);
  const bool live = (int)e < n;
  auto ld = [&](int k) -> double { return (double)rowld(F, k, n, e); };
  double inv_det = 1.0;
  if constexpr (Z::GEO) {
    if (live) inv_det = 1.0 / (double)rowld(m.detJ, 0, n, e);
  }
  for (int r = w; r < Z::BS; r += NW) {
    double v = 0.0;
    if (live) {
      v = (double)rowld(x, r, n, e);
      if (r >= Z::NV) {
        if constexpr (Z::GEO) {
          if (!row_unused<D, T>(m, r / Z::NP, r % Z::NP)) v *= inv_det;
        } else {
          v *= ld(Z::OD + r - Z::NV);
        }
      }
    }
    xs[r][lane] = v;
  }
  __syncthreads();
  for (int u = w; u < Z::NU; u += NW) {
    double s = xs[Z::NP + u][lane];
    if (live) {
#pragma unroll
      for (int k = 0; k < Z::NE; ++k) s -= ld(Z::OG + u * Z::NE + k) * xs[Z::NV + k][lane];
    }
    xs[Z::NP + u][lane] = s;
  }
  __syncthreads();
  const double sg = scale();
  constexpr int NVW = (Z::NV + NW - 1) / NW;
  double z[NVW];
#pragma unroll
  for (int i = 0; i < NVW; ++i) {
    const int v = w + NW * i;
    double s = 0.0;
    if (v < Z::NV && live) {
#pragma unroll
      for (int c = 0; c < Z::NV; ++c) s += ld(Z::OS + v * Z::NV + c) * xs[c][lane];
      rowref(y, v, n, e) = (T)(sg * s);
    }
    z[i] = s;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NVW; ++i) {
    const int v = w + NW * i;
    if (v >= Z::NP && v < Z::NV) xs[v][lane] = z[i];
  }
  __syncthreads();
  if (!live) return;
  if constexpr (Z::GEO) {
    static_assert(D * D == NW, "one stress field per wave");
    const Tab<2, P, T>& tb = tab<2, P, T>();
    const int fe = 3 + w, b = w >> 1, a = w & 1;
    double zq[S::NQ], zf[3][S::NFQ][2];
#pragma unroll
    for (int q = 0; q < S::NQ; ++q) zq[q] = 0.0;
#pragma unroll
    for (int fc = 0; fc < 3; ++fc)
#pragma unroll
      for (int rr = 0; rr < S::NFQ; ++rr) zf[fc][rr][0] = zf[fc][rr][1] = 0.0;
    // (j rolled: one mode's table entries live at a time)
#pragma unroll 1
    for (int j = 0; j < S::NP; ++j) {
      if (row_unused<D, T>(m, 1, j)) continue;  // (the two velocity fields share their order)
      const double z0 = xs[S::NP + j][lane], z1 = xs[2 * S::NP + j][lane];
      const double zb = b == 0 ? z0 : z1;
#pragma unroll
      for (int q = 0; q < S::NQ; ++q) zq[q] += (double)tb.phi[q][j] * zb;
#pragma unroll
      for (int fc = 0; fc < 3; ++fc)
#pragma unroll
        for (int rr = 0; rr < S::NFQ; ++rr) {
          zf[fc][rr][0] += (double)tb.fphi[fc][rr][j] * z0;
          zf[fc][rr][1] += (double)tb.fphi[fc][rr][j] * z1;
        }
    }
    schur_geo_rows<P, T>(tb, m, bc, e, b, a, zq, zf, [&](int k, double hzk) {
      const int row = fe * S::NP + k;
      double s = xs[row][lane];
      if (!row_unused<D, T>(m, fe, k)) s -= hzk;
      rowref(y, row, n, e) = (T)(sg * s);
    });
  } else {
    for (int k = w; k < Z::NE; k += NW) {
      double s = xs[Z::NV + k][lane];
#pragma unroll
      for (int c = 0; c < Z::NU; ++c) s -= ld(Z::OH + k * Z::NU + c) * xs[Z::NP + c][lane];
      rowref(y, Z::NV + k, n, e) = (T)(sg * s);
    }
  }
}

template <int D, int P, class T>
__global__ void __launch_bounds__(256) k_schur_apply(const float* __restrict__ F, const T* __restrict__ x,
                                                      T* __restrict__ y, MeshView<T> m, int bc) {
  schur_apply_tile<D, P, T>(F, x, y, m, bc, (int)blockIdx.x * kPrecEB, [] { return 1.0; });
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
