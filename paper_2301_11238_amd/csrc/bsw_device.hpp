// Device-side building blocks: shapes, constant-memory reference tables,
// pointwise physics of the regularised-Bingham shallow-water system and its
// tangent.  Paper references: Sec. 3 (Eqs. Uterm, Fterm, Qterm, Sterm, Gterm),
// Sec. 4 (regularisations), Sec. 5 (Eq. HLLSolver, central fluxes, Sec. 5.2
// boundary states) and Appendix A (tangent terms).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bsw {

template <int D, int P>
struct Shape {
  static constexpr int NP = D == 1 ? P + 1 : (P + 1) * (P + 2) / 2;
  static constexpr int NQ = D == 1 ? P + 1 : (P == 1 ? 3 : (P == 2 ? 7 : 12));
  static constexpr int NFQ = D == 1 ? 1 : P + 1;
  static constexpr int NFC = D + 1;
  static constexpr int NF = 1 + D + D * D;
  static constexpr int NV = 1 + D;
  static constexpr int BS = NF * NP;
};

template <int D, int P, class T>
struct Tab {
  using S = Shape<D, P>;
  T phi[S::NQ][S::NP];
  T dphi[S::NQ][S::NP][D];
  T qw[S::NQ];
  T fphi[S::NFC][S::NFQ][S::NP];
  T fw[S::NFQ];
};

// All (dim, order, precision) combinations the library supports share one
// constant-memory block; each gets a fixed, 16-byte aligned slot.
constexpr int kNumCombos = 8;
constexpr int kCombo[kNumCombos][2] = {{1, 0}, {1, 1}, {1, 2}, {1, 3}, {1, 4}, {2, 1}, {2, 2}, {2, 3}};

template <class T>
constexpr size_t tab_bytes_rt(int D, int P) {
  const int NP = D == 1 ? P + 1 : (P + 1) * (P + 2) / 2;
  const int NQ = D == 1 ? P + 1 : (P == 1 ? 3 : (P == 2 ? 7 : 12));
  const int NFQ = D == 1 ? 1 : P + 1;
  const int NFC = D + 1;
  return sizeof(T) * (size_t)(NQ * NP + NQ * NP * D + NQ + NFC * NFQ * NP + NFQ);
}
constexpr size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// slot order: all double tables, then all float tables
constexpr size_t tab_offset_rt(int D, int P, bool is_float) {
  size_t off = 0;
  for (int pass = 0; pass < 2; ++pass)
    for (int k = 0; k < kNumCombos; ++k) {
      if (pass == (is_float ? 1 : 0) && kCombo[k][0] == D && kCombo[k][1] == P) return off;
      off += align16(pass == 0 ? tab_bytes_rt<double>(kCombo[k][0], kCombo[k][1])
                               : tab_bytes_rt<float>(kCombo[k][0], kCombo[k][1]));
    }
  return off;
}
constexpr size_t kTabBytesTotal = tab_offset_rt(99, 99, true);

template <class T>
struct DevParams {
  T g, gc, gs, rho_inv, eta, s0, gam, bet, inv_dt;
  int reg, bc, jfrozen;
  const T* dirtab;  // device [4][7]: Dirichlet exterior states of boundary tags 0..3
};

template <class T>
struct MeshView {
  int n_el;
  const T* dxi;      // [D*D][n_el] : d xi_r / d x_a stored at r*D + a
  const T* detJ;     // [n_el]
  const T* nrm;      // [NFC*D][n_el]
  const T* hlen;     // [NFC][n_el] : face length / 2 (2-D), 1 (1-D)
  const int* nbr;    // [NFC][n_el] : 4*neighbour + neighbour's local face; on the boundary
                     // -1 - code, code = kind | tag << 2 (kind 0: the parameters' bc)
  const double* vert;  // [(D+1)*D][n_el] vertex coordinates (FP64)
  const T* bed;        // [NP][n_el] modal coefficients of the bed H; nullptr = flat bed
  int nmodes;          // modes used by h | u << 8 | E << 16 (orders m1, m2, m3; NP when uniform)
};

template <class T> __device__ __forceinline__ T dsqrt(T x);
template <> __device__ __forceinline__ double dsqrt<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float dsqrt<float>(float x) { return sqrtf(x); }
template <class T> __device__ __forceinline__ T dtanh(T x);
template <> __device__ __forceinline__ double dtanh<double>(double x) { return tanh(x); }
template <> __device__ __forceinline__ float dtanh<float>(float x) { return tanhf(x); }

// ------------------------------------------------------------------ state at a point
template <int D, class T>
struct Pt {
  T h;
  T u[D];
  T E[D][D];  // E[a][b] = d u_b / d x_a
};

template <int D, class T>
__device__ __forceinline__ void unpack(const T* X, Pt<D, T>& s) {
  s.h = X[0];
#pragma unroll
  for (int b = 0; b < D; ++b) s.u[b] = X[1 + b];
#pragma unroll
  for (int b = 0; b < D; ++b)
#pragma unroll
    for (int a = 0; a < D; ++a) s.E[a][b] = X[1 + D + b * D + a];
}

// --------------------------------------------------------------- constitutive law (Sec. 4)
// 2-D reading of the regularisations: sigma = (2 eta + psi(s)) (D + tr(D) I),
// s = ||D||_c / sqrt(2); psi is the paper's 1-D sigma_B^k evaluated at the shear
// rate s and divided by 2 s.  Also returns q = psi'(s) / (2 s), finite at s = 0.
// The reg-3 small-shear branch runs in FP64 whatever T is.
template <class T>
__device__ __forceinline__ void psi_q(const DevParams<T>& p, T s, T& psi, T& q) {
  if (p.s0 == T(0)) { psi = T(0); q = T(0); return; }
  if (p.reg == 1) {
    const T h = T(0.5) / p.bet;
    const T x = p.gam * s - p.s0;
    T m, dm;
    if (x >= h) { m = x; dm = T(1); }
    else if (x <= -h) { m = T(0); dm = T(0); }
    else { const T y = x + h; m = T(0.5) * p.bet * y * y; dm = p.bet * y; }
    const T den = p.s0 + m;
    psi = p.s0 * p.gam / den;
    q = (dm == T(0)) ? T(0) : -(p.s0 * p.gam * p.gam * dm) / (den * den) / (T(2) * s);
  } else if (p.reg == 2) {
    const T h = T(0.5) / p.bet;
    const T y = p.gam * s;
    if (y >= p.s0 + h) {
      psi = p.s0 / s;
      q = -p.s0 / (T(2) * s * s * s);
    } else if (y >= p.s0 - h) {
      const T z = p.s0 - y + h;
      const T num = T(2) * p.s0 - p.bet * z * z;
      psi = num / (T(2) * s);
      q = (p.bet * z * p.gam / s - num / (T(2) * s * s)) / (T(2) * s);
    } else {
      psi = p.gam;
      q = T(0);
    }
  } else {
    const double x = (double)p.gam * (double)s;
    const double sg = (double)p.s0 * (double)p.gam;
    double ps, r;
    if (x < 1e-2) {
      const double x2 = x * x;
      // tanh(x)/x and (x sech^2 x - tanh x)/x^3 by their Taylor series
      ps = 1.0 + x2 * (-1.0 / 3.0 + x2 * (2.0 / 15.0 + x2 * (-17.0 / 315.0)));
      r = -2.0 / 3.0 + x2 * (8.0 / 15.0 + x2 * (-34.0 / 105.0 + x2 * (496.0 / 2835.0)));
    } else {
      const double t = tanh(x);
      ps = t / x;
      r = (x * (1.0 - t * t) - t) / (x * x * x);
    }
    psi = (T)(sg * ps);
    q = (T)(0.5 * sg * (double)p.gam * (double)p.gam * r);
  }
}

template <int D, class T>
struct Stress {
  T sig[D][D];
  T Tm[D][D];  // D + tr(D) I
  T mu;        // 2 eta + psi
  T q;         // psi'(s) / (2 s)
};

template <int D, class T>
__device__ __forceinline__ void stress(const DevParams<T>& p, const T (&E)[D][D], Stress<D, T>& st) {
  T tr = T(0);
#pragma unroll
  for (int a = 0; a < D; ++a) tr += E[a][a];
  T n2 = tr * tr;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const T dab = T(0.5) * (E[a][b] + E[b][a]);
      n2 += dab * dab;
      st.Tm[a][b] = dab + (a == b ? tr : T(0));
    }
  const T s = dsqrt(T(0.5) * n2);
  T psi, q;
  psi_q(p, s, psi, q);
  st.mu = T(2) * p.eta + psi;
  st.q = q;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) st.sig[a][b] = st.mu * st.Tm[a][b];
}

// d sigma = mu (dD + tr(dD) I) + q (T : dE) T   (chain rule of the law above)
template <int D, class T>
__device__ __forceinline__ void stress_tan(const Stress<D, T>& st, const T (&dE)[D][D], T (&dsig)[D][D]) {
  T tr = T(0), td = T(0);
#pragma unroll
  for (int a = 0; a < D; ++a) tr += dE[a][a];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) td += st.Tm[a][b] * dE[a][b];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const T ddab = T(0.5) * (dE[a][b] + dE[b][a]) + (a == b ? tr : T(0));
      dsig[a][b] = st.mu * ddab + st.q * td * st.Tm[a][b];
    }
}

// ----------------------------------------------------------------- boundary states (Sec. 5.2)
template <int D, class T>
__device__ __forceinline__ void mirror(const T* n, const Pt<D, T>& in, Pt<D, T>& out) {
  T R[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) R[a][b] = (a == b ? T(1) : T(0)) - T(2) * n[a] * n[b];
  out.h = in.h;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    T s = T(0);
#pragma unroll
    for (int b = 0; b < D; ++b) s += R[a][b] * in.u[b];
    out.u[a] = s;
  }
  T RE[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int d = 0; d < D; ++d) {
      T s = T(0);
#pragma unroll
      for (int c = 0; c < D; ++c) s += R[a][c] * in.E[c][d];
      RE[a][d] = s;
    }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T s = T(0);
#pragma unroll
      for (int d = 0; d < D; ++d) s += RE[a][d] * R[d][b];
      out.E[a][b] = s;
    }
}

// Exterior state of a boundary face with code = kind | tag << 2 (Sec. 5.2):
// kind 1 wall, 2 Neumann, 3 Dirichlet, 0 the parameters' bc; a Dirichlet face
// reads its tag's state from a small device table when it needs it (kept out
// of the kernel's uniform registers).  For the tangent, din -> dout
// (Dirichlet: zero).
template <int D, class T>
__device__ __forceinline__ void exterior(const DevParams<T>& p, const T* n, int code, const Pt<D, T>& in,
                                         Pt<D, T>& out) {
  const int kind = (code & 3) ? (code & 3) : p.bc;
  if (kind == 1) mirror<D, T>(n, in, out);
  else if (kind == 2) out = in;
  else {
    unpack<D, T>(p.dirtab + 7 * (code >> 2), out);
  }
}
template <int D, class T>
__device__ __forceinline__ void exterior_tan(const DevParams<T>& p, const T* n, int code, const Pt<D, T>& din,
                                             Pt<D, T>& dout) {
  const int kind = (code & 3) ? (code & 3) : p.bc;
  if (kind == 1) mirror<D, T>(n, din, dout);
  else if (kind == 2) dout = din;
  else {
    dout.h = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      dout.u[a] = T(0);
#pragma unroll
      for (int b = 0; b < D; ++b) dout.E[a][b] = T(0);
    }
  }
}

// ------------------------------------------------------------------ HLL (Eq. HLLSolver)
// Normal flux A(V; n) = sum_a F_a n_a (Eq. Fterm) and conserved U (Eq. Uterm).
template <int D, class T>
__device__ __forceinline__ void nflux(T gc, const Pt<D, T>& s, const T* n, T& un, T (&A)[1 + D], T (&U)[1 + D]) {
  un = T(0);
#pragma unroll
  for (int a = 0; a < D; ++a) un += s.u[a] * n[a];
  const T hun = s.h * un;
  const T pr = T(0.5) * gc * s.h * s.h;
  A[0] = hun;
  U[0] = s.h;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    A[1 + b] = hun * s.u[b] + pr * n[b];
    U[1 + b] = s.h * s.u[b];
  }
}

template <int D, class T>
struct HLLState {
  T Am[1 + D], Um[1 + D], Ap[1 + D], Up[1 + D];
  T unm, unp, cm, cp, SL, SR;
  bool left_m, right_m;  // which side sets S_L / S_R (ties -> own side)
  int branch;            // 0: A(U-), 1: mixed, 2: A(U+)
};

template <int D, class T>
__device__ __forceinline__ void hll(const DevParams<T>& p, const Pt<D, T>& m, const Pt<D, T>& pl, const T* n,
                                    HLLState<D, T>& H, T (&F)[1 + D]) {
  nflux<D, T>(p.gc, m, n, H.unm, H.Am, H.Um);
  nflux<D, T>(p.gc, pl, n, H.unp, H.Ap, H.Up);
  H.cm = dsqrt(p.g * m.h);
  H.cp = dsqrt(p.g * pl.h);
  const T l1 = H.unm - H.cm, l2 = H.unp - H.cp, r1 = H.unm + H.cm, r2 = H.unp + H.cp;
  H.left_m = l1 <= l2;
  H.right_m = r1 >= r2;
  H.SL = H.left_m ? l1 : l2;
  H.SR = H.right_m ? r1 : r2;
  if (H.SL >= T(0)) {
    H.branch = 0;
#pragma unroll
    for (int k = 0; k <= D; ++k) F[k] = H.Am[k];
  } else if (H.SR <= T(0)) {
    H.branch = 2;
#pragma unroll
    for (int k = 0; k <= D; ++k) F[k] = H.Ap[k];
  } else {
    H.branch = 1;
    const T inv = T(1) / (H.SR - H.SL);
    const T slsr = H.SL * H.SR;
#pragma unroll
    for (int k = 0; k <= D; ++k) F[k] = (H.SR * H.Am[k] - H.SL * H.Ap[k] + slsr * (H.Up[k] - H.Um[k])) * inv;
  }
}

template <int D, class T>
__device__ __forceinline__ void nflux_tan(T gc, const Pt<D, T>& s, const Pt<D, T>& ds, const T* n, T un,
                                          T& dun, T (&dA)[1 + D], T (&dU)[1 + D]) {
  dun = T(0);
#pragma unroll
  for (int a = 0; a < D; ++a) dun += ds.u[a] * n[a];
  const T dhun = ds.h * un + s.h * dun;
  dA[0] = dhun;
  dU[0] = ds.h;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    dA[1 + b] = dhun * s.u[b] + s.h * un * ds.u[b] + gc * s.h * ds.h * n[b];
    dU[1 + b] = ds.h * s.u[b] + s.h * ds.u[b];
  }
}

// exact directional derivative of the HLL flux (wave speeds included)
template <int D, class T>
__device__ __forceinline__ void hll_tan(const DevParams<T>& p, const HLLState<D, T>& H, const Pt<D, T>& m,
                                        const Pt<D, T>& pl, const Pt<D, T>& dm, const Pt<D, T>& dp, const T* n,
                                        T (&dF)[1 + D]) {
  T dunm, dunp, dAm[1 + D], dUm[1 + D], dAp[1 + D], dUp[1 + D];
  nflux_tan<D, T>(p.gc, m, dm, n, H.unm, dunm, dAm, dUm);
  nflux_tan<D, T>(p.gc, pl, dp, n, H.unp, dunp, dAp, dUp);
  if (H.branch == 0) {
#pragma unroll
    for (int k = 0; k <= D; ++k) dF[k] = dAm[k];
    return;
  }
  if (H.branch == 2) {
#pragma unroll
    for (int k = 0; k <= D; ++k) dF[k] = dAp[k];
    return;
  }
  const T dcm = T(0.5) * p.g * dm.h / H.cm;
  const T dcp = T(0.5) * p.g * dp.h / H.cp;
  // exact wave-speed derivatives, or none (the paper's frozen-speed form)
  const T dSL = p.jfrozen ? T(0) : (H.left_m ? dunm - dcm : dunp - dcp);
  const T dSR = p.jfrozen ? T(0) : (H.right_m ? dunm + dcm : dunp + dcp);
  const T inv = T(1) / (H.SR - H.SL);
  const T slsr = H.SL * H.SR;
  const T dslsr = dSL * H.SR + H.SL * dSR;
#pragma unroll
  for (int k = 0; k <= D; ++k) {
    const T jump = H.Up[k] - H.Um[k];
    const T num = H.SR * H.Am[k] - H.SL * H.Ap[k] + slsr * jump;
    const T dnum = dSR * H.Am[k] + H.SR * dAm[k] - dSL * H.Ap[k] - H.SL * dAp[k] + dslsr * jump +
                   slsr * (dUp[k] - dUm[k]);
    dF[k] = (dnum - num * (dSR - dSL) * inv) * inv;
  }
}

}  // namespace bsw
