// Element pass on triangles with one lane per element: the residual of
// Eq. WeakForm7 (MODE 0) and its directional derivative along x (MODE 1,
// Appendix A).
//
// A workgroup of NW waves takes a tile of 64 consecutive elements; lane l of
// every wave works on element e0 + l.  The waves split the work into units
// that are the same for all 64 elements (a face chunk, a volume point, an
// output field group), so a wave reads the reference tables at wave-uniform
// indices (through the scalar unit) and every coefficient load is one
// coalesced 64-element row.  Per tile:
//   1. face integrands: each wave evaluates the points of its face chunks:
//      the element's side from its coefficients, the neighbour's side from
//      the neighbour's coefficients (its local face differs from lane to
//      lane, so that table is read per lane) or, for the linearisation state
//      of MODE 1, from the stored traces; HLL flux, central stress and
//      velocity fluxes, boundary states.  Integrands go to LDS.
//   2. each wave lifts the face integrands of its output fields (registers);
//   3. volume integrands: each wave interpolates W (and x) at its volume
//      points, loading every coefficient row once for all of them, and
//      evaluates fluxes, Bingham stress and source.  Integrands go to LDS
//      (the same buffer).
//   4. each wave contracts the volume integrands of its fields with the test
//      functions, adds the mass terms, subtracts b_old (MODE 0) and writes its
//      rows.
// Mass terms: the element rules integrate products of two basis functions
// exactly and the basis is orthonormal, so <phi_i, h>_e / dt = |J| h_i / dt
// and <phi_i, E>_e = |J| E_i are taken from the coefficients.
#pragma once
#include "bsw_kernels.hpp"

namespace bsw {

template <int P, class T, int MODE, int NW>
struct E2 {
  using S = Shape<2, P>;
  static constexpr int EB = 64;                               // elements per tile
  static constexpr int NT = 64 * NW;                          // lanes per workgroup
  static constexpr int NFP = S::NFC * S::NFQ;                 // face points per element
  static constexpr int NVI = 10;                              // volume integrands per point
  static constexpr int NFI = 5;                               // face integrands per point
  static constexpr int QW = (S::NQ + NW - 1) / NW;            // volume points per wave
  static constexpr int PC = P < 3 ? S::NFQ : 2;               // face points per chunk (register budget)
  static constexpr int NCH = (S::NFQ + PC - 1) / PC;          // chunks per face
  static constexpr int GS = (Shape<2, P>::NF + NW - 1) / NW;  // output fields per wave
  static constexpr int LDS = (S::NQ * NVI > NFP * NFI ? S::NQ * NVI : NFP * NFI) * EB;
};

// Volume integrands at one point (weight wq = w_q |J|), besides the mass
// terms: o[b] = wq (h u_b / dt + sl_b h) (b = 0, 1; with the source slope sl),
// o[2 + r*3 + f] = -wq sum_a xi_ra (F_a - Q_a)_f, o[8 + b] = wq u_b.
template <class T>
__device__ __forceinline__ void e2_vol(const DevParams<T>& p, const Geo<2, T>& g, T wq, const Pt<2, T>& s,
                                       const Stress<2, T>& st, const T (&sl)[2], T (&o)[10]) {
  T G[2][3];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const T hua = s.h * s.u[a];
    G[a][0] = hua;
#pragma unroll
    for (int b = 0; b < 2; ++b)
      G[a][1 + b] = hua * s.u[b] + (a == b ? T(0.5) * p.gc * s.h * s.h : T(0)) - s.h * st.sig[b][a] * p.rho_inv;
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) o[b] = wq * (s.h * s.u[b] * p.inv_dt + sl[b] * s.h);
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int f = 0; f < 3; ++f) o[2 + r * 3 + f] = -wq * (g.xi[r][0] * G[0][f] + g.xi[r][1] * G[1][f]);
#pragma unroll
  for (int b = 0; b < 2; ++b) o[8 + b] = wq * s.u[b];
}

// its directional derivative along ds at the state s
template <class T>
__device__ __forceinline__ void e2_vol_tan(const DevParams<T>& p, const Geo<2, T>& g, T wq, const Pt<2, T>& s,
                                           const Stress<2, T>& st, const Pt<2, T>& ds, const T (&sl)[2],
                                           T (&o)[10]) {
  T dsig[2][2];
  stress_tan<2, T>(st, ds.E, dsig);
  T G[2][3];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const T hua = s.h * s.u[a];
    const T dhua = ds.h * s.u[a] + s.h * ds.u[a];
    G[a][0] = dhua;
#pragma unroll
    for (int b = 0; b < 2; ++b)
      G[a][1 + b] = dhua * s.u[b] + hua * ds.u[b] + (a == b ? p.gc * s.h * ds.h : T(0)) -
                    (ds.h * st.sig[b][a] + s.h * dsig[b][a]) * p.rho_inv;
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) o[b] = wq * ((ds.h * s.u[b] + s.h * ds.u[b]) * p.inv_dt + sl[b] * ds.h);
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int f = 0; f < 3; ++f) o[2 + r * 3 + f] = -wq * (g.xi[r][0] * G[0][f] + g.xi[r][1] * G[1][f]);
#pragma unroll
  for (int b = 0; b < 2; ++b) o[8 + b] = wq * ds.u[b];
}

// Face integrands at one point (weight wr = w_r |face| / 2):
// o[f] = wr (F_hll . n - Q_central . n)_f (f = 0..2), o[3 + b] = -wr (u_b- + u_b+) / 2;
// the lift multiplies o[3 + b] by n_a for the gradient row (b, a).
template <class T>
__device__ __forceinline__ void e2_face(const DevParams<T>& p, const T* n, T wr, const Pt<2, T>& sm,
                                        const Pt<2, T>& sp, T (&o)[5]) {
  HLLState<2, T> H;
  T Fn[3];
  hll<2, T>(p, sm, sp, n, H, Fn);
  Stress<2, T> qm, qp;
  stress<2, T>(p, sm.E, qm);
  stress<2, T>(p, sp.E, qp);
  o[0] = wr * Fn[0];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    T qn = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a) qn += (sm.h * qm.sig[b][a] + sp.h * qp.sig[b][a]) * n[a];
    o[1 + b] = wr * (Fn[1 + b] - T(0.5) * qn * p.rho_inv);
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) o[3 + b] = -wr * T(0.5) * (sm.u[b] + sp.u[b]);
}

template <class T>
__device__ __forceinline__ void e2_face_tan(const DevParams<T>& p, const T* n, T wr, const Pt<2, T>& sm,
                                            const Pt<2, T>& sp, const Pt<2, T>& dsm, const Pt<2, T>& dsp,
                                            T (&o)[5]) {
  HLLState<2, T> H;
  T Fn[3], dFn[3];
  hll<2, T>(p, sm, sp, n, H, Fn);
  hll_tan<2, T>(p, H, sm, sp, dsm, dsp, n, dFn);
  Stress<2, T> qm, qp;
  stress<2, T>(p, sm.E, qm);
  stress<2, T>(p, sp.E, qp);
  T dsm_sig[2][2], dsp_sig[2][2];
  stress_tan<2, T>(qm, dsm.E, dsm_sig);
  stress_tan<2, T>(qp, dsp.E, dsp_sig);
  o[0] = wr * dFn[0];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    T qn = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
      qn += (dsm.h * qm.sig[b][a] + sm.h * dsm_sig[b][a] + dsp.h * qp.sig[b][a] + sp.h * dsp_sig[b][a]) * n[a];
    o[1 + b] = wr * (dFn[1 + b] - T(0.5) * qn * p.rho_inv);
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) o[3 + b] = -wr * T(0.5) * (dsm.u[b] + dsp.u[b]);
}

// Output field f of a wave: 0 h, 1 u1, 2 u2 (balance rows) or 3 + 2b + a,
// the gradient row (b, a) (E_ab = d u_b / d x_a, Eq. gradientVel).  Each wave
// owns the fields w, w + NW, ...; acc[s][i] holds row i of its s-th field.

// lift of the face integrands of field f (stage 2): integrand f of a face
// point is the flux of balance field f, or for the gradient row (b, a) the
// integrand 3 + b, -wr (u_b- + u_b+) / 2, times n_a of the point's face
template <int P, class T>
__device__ __forceinline__ void e2_lift_faces(const Tab<2, P, T>& tb, const T* sI, int lane, int f,
                                              const T (&nv)[3][2], T (&acc)[Shape<2, P>::NP]) {
  using S = Shape<2, P>;
  constexpr int EB = 64;
  const int k = f < 3 ? f : 3 + ((f - 3) >> 1);
  const int a = (f - 3) & 1;
#pragma unroll
  for (int fc = 0; fc < S::NFC; ++fc) {
    const T sc = f < 3 ? T(1) : (a == 0 ? nv[fc][0] : nv[fc][1]);
#pragma unroll 1
    for (int rr = 0; rr < S::NFQ; ++rr) {
      const T v = sI[(size_t)((fc * S::NFQ + rr) * 5 + k) * EB + lane] * sc;
#pragma unroll
      for (int i = 0; i < S::NP; ++i) acc[i] += tb.fphi[fc][rr][i] * v;
    }
  }
}

// contraction of the volume integrands of field f with the test functions
// (stage 4)
template <int P, class T>
__device__ __forceinline__ void e2_contract_volume(const Tab<2, P, T>& tb, const T* sI, int lane, int f,
                                                   const Geo<2, T>& geo, T (&acc)[Shape<2, P>::NP]) {
  using S = Shape<2, P>;
  constexpr int EB = 64;
  if (f < 3) {
#pragma unroll 1
    for (int q = 0; q < S::NQ; ++q) {
      const T* o = sI + (size_t)q * 10 * EB + lane;
      const T b0 = o[(2 + f) * EB], b1 = o[(5 + f) * EB];
      const T av = f == 0 ? T(0) : o[(f - 1) * EB];
#pragma unroll
      for (int i = 0; i < S::NP; ++i) acc[i] += tb.phi[q][i] * av + tb.dphi[q][i][0] * b0 + tb.dphi[q][i][1] * b1;
    }
  } else {
    // row (b, a): sum_q sum_r dphi_qir xi_ra wq u_b = sum_r xi_ra (sum_q dphi_qir wq u_b)
    const int b = (f - 3) >> 1, a = (f - 3) & 1;
    T t0[S::NP], t1[S::NP];
#pragma unroll
    for (int i = 0; i < S::NP; ++i) t0[i] = t1[i] = T(0);
#pragma unroll 1
    for (int q = 0; q < S::NQ; ++q) {
      const T wu = sI[(size_t)(q * 10 + 8 + b) * EB + lane];
#pragma unroll
      for (int i = 0; i < S::NP; ++i) {
        t0[i] += tb.dphi[q][i][0] * wu;
        t1[i] += tb.dphi[q][i][1] * wu;
      }
    }
    const T x0 = a == 0 ? geo.xi[0][0] : geo.xi[0][1];
    const T x1 = a == 0 ? geo.xi[1][0] : geo.xi[1][1];
#pragma unroll
    for (int i = 0; i < S::NP; ++i) acc[i] += x0 * t0[i] + x1 * t1[i];
  }
}

template <int P, class T, int MODE, int NW>
__device__ __forceinline__ void elem2_tile(const T* __restrict__ W, const T* __restrict__ x,
                                           const T* __restrict__ bold, T* __restrict__ out,
                                           const T* __restrict__ trW, const MeshView<T>& m, const DevParams<T>& p,
                                           int e0) {
  using S = Shape<2, P>;
  using C = E2<P, T, MODE, NW>;
  constexpr int EB = C::EB;
  constexpr bool TAN = MODE == 1;
  const Tab<2, P, T>& tb = tab<2, P, T>();
  const int n = m.n_el;
  const int lane = (int)threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int e = e0 + lane;
  const bool live = e < n;
  const unsigned ec = live ? e : n - 1;  // dead lanes of a ragged tail read a valid element
  __shared__ T sI[C::LDS];

  // -------------------------------------------------- stage 1: face integrands
  for (int u = w; u < S::NFC * C::NCH; u += NW) {
    const int fc = u / C::NCH, r0 = (u % C::NCH) * C::PC;
    const int code = rowld(m.nbr, fc, n, ec);
    const bool inner = code >= 0;
    const unsigned nb = inner ? (unsigned)(code >> 2) : ec;
    const int gf = inner ? (code & 3) : 0;
    T nvec[2];
    nvec[0] = rowld(m.nrm, fc * 2 + 0, n, ec);
    nvec[1] = rowld(m.nrm, fc * 2 + 1, n, ec);
    const T hl = rowld(m.hlen, fc, n, ec);
    // the neighbour's basis at its own face points, per lane (point order
    // reversed along the shared edge)
    T tnb[C::PC][S::NP];
#pragma unroll
    for (int j = 0; j < C::PC; ++j) {
      const int rr = r0 + j < S::NFQ ? r0 + j : S::NFQ - 1;
#pragma unroll
      for (int i = 0; i < S::NP; ++i) tnb[j][i] = tb.fphi[gf][S::NFQ - 1 - rr][i];
    }
    T Xm[C::PC][S::NF], Xp[C::PC][S::NF], dXm[TAN ? C::PC : 1][S::NF], dXp[TAN ? C::PC : 1][S::NF];
    // one field at a time (a rolled loop: unrolled, every field's coefficient
    // loads would be hoisted together and exhaust the registers); the field
    // index is wave-uniform, so placing the values is a scalar branch
#pragma unroll 1
    for (int f = 0; f < S::NF; ++f) {
      // residual: the element's and the neighbour's side of W from their
      // coefficients; Jacobian: those of x from their coefficients, those of
      // the linearisation state W from its stored traces (below)
      const T* __restrict__ A = TAN ? x : W;
      T c[S::NP], cn[S::NP];
#pragma unroll
      for (int i = 0; i < S::NP; ++i) {
        c[i] = rowld(A, f * S::NP + i, n, ec);
        cn[i] = rowld(A, f * S::NP + i, n, nb);
      }
#pragma unroll
      for (int j = 0; j < C::PC; ++j) {
        const int rr = r0 + j < S::NFQ ? r0 + j : S::NFQ - 1;
        T s1 = T(0), s2 = T(0);
#pragma unroll
        for (int i = 0; i < S::NP; ++i) {
          s1 += tb.fphi[fc][rr][i] * c[i];
          s2 += tnb[j][i] * cn[i];
        }
#pragma unroll
        for (int ff = 0; ff < S::NF; ++ff)
          if (ff == f) {
            if constexpr (!TAN) { Xm[j][ff] = s1; Xp[j][ff] = s2; }
            else { dXm[j][ff] = s1; dXp[j][ff] = s2; }
          }
      }
    }
#pragma unroll
    for (int j = 0; j < C::PC; ++j) {
      const int rr = r0 + j;
      if (rr >= S::NFQ) break;
      if constexpr (TAN) {
        // both sides of the linearisation state from its traces
#pragma unroll
        for (int f = 0; f < S::NF; ++f) {
          Xm[j][f] = rowld(trW, f * C::NFP + fc * S::NFQ + rr, n, ec);
          Xp[j][f] = rowld(trW, f * C::NFP + (S::NFQ - 1 - rr), n, (unsigned)(gf * S::NFQ) * (unsigned)n + nb);
        }
      }
      Pt<2, T> sm, sp, dsm, dsp;
      unpack<2, T>(Xm[j], sm);
      unpack<2, T>(Xp[j], sp);
      if constexpr (TAN) {
        unpack<2, T>(dXm[j], dsm);
        unpack<2, T>(dXp[j], dsp);
      }
      if (!inner) {
        exterior<2, T>(p, nvec, -1 - code, sm, sp);
        if constexpr (TAN) exterior_tan<2, T>(p, nvec, -1 - code, dsm, dsp);
      }
      T o[5];
      const T wr = tb.fw[rr] * hl;
      if constexpr (TAN) e2_face_tan<T>(p, nvec, wr, sm, sp, dsm, dsp, o);
      else e2_face<T>(p, nvec, wr, sm, sp, o);
      T* dst = sI + (size_t)(fc * S::NFQ + rr) * 5 * EB + lane;
#pragma unroll
      for (int k = 0; k < 5; ++k) dst[k * EB] = o[k];
      // points one after the other (interleaving their flux evaluations
      // would multiply the live registers)
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();

  // -------------------------------------------------- stage 2: face lift
  T acc[C::GS][S::NP];
#pragma unroll
  for (int s = 0; s < C::GS; ++s)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) acc[s][i] = T(0);
  {
    T nv[3][2];
#pragma unroll
    for (int fc = 0; fc < 3; ++fc)
#pragma unroll
      for (int a = 0; a < 2; ++a) nv[fc][a] = rowld(m.nrm, fc * 2 + a, n, ec);
#pragma unroll
    for (int s = 0; s < C::GS; ++s) {
      const int f = w + s * NW;
      if (f < S::NF) e2_lift_faces<P, T>(tb, sI, lane, f, nv, acc[s]);
    }
  }
  __syncthreads();

  // -------------------------------------------------- stage 3: volume integrands
  Geo<2, T> geo;
  load_geo<2, T>(m, ec, geo);
  {
    T X[C::QW][S::NF], dX[TAN ? C::QW : 1][S::NF];
#pragma unroll 1
    for (int f = 0; f < S::NF; ++f) {
      T c[S::NP], cx[TAN ? S::NP : 1];
#pragma unroll
      for (int i = 0; i < S::NP; ++i) {
        c[i] = rowld(W, f * S::NP + i, n, ec);
        if constexpr (TAN) cx[i] = rowld(x, f * S::NP + i, n, ec);
      }
      // the mass terms of the wave's own rows of field f: |J| h_i / dt on the
      // depth rows, |J| E_i on the gradient rows (of the pass's argument)
#pragma unroll
      for (int s = 0; s < C::GS; ++s) {
        if (w + s * NW != f || (f != 0 && f < 3)) continue;
        const T sc = f == 0 ? geo.detJ * p.inv_dt : geo.detJ;
#pragma unroll
        for (int i = 0; i < S::NP; ++i) acc[s][i] += sc * (TAN ? cx[i] : c[i]);
      }
#pragma unroll
      for (int j = 0; j < C::QW; ++j) {
        const int q = w + j * NW < S::NQ ? w + j * NW : S::NQ - 1;
        T s1 = T(0), s2 = T(0);
#pragma unroll
        for (int i = 0; i < S::NP; ++i) {
          s1 += tb.phi[q][i] * c[i];
          if constexpr (TAN) s2 += tb.phi[q][i] * cx[i];
        }
#pragma unroll
        for (int ff = 0; ff < S::NF; ++ff)
          if (ff == f) {
            X[j][ff] = s1;
            if constexpr (TAN) dX[j][ff] = s2;
          }
      }
    }
#pragma unroll
    for (int j = 0; j < C::QW; ++j) {
      const int q = w + j * NW;
      if (q >= S::NQ) break;
      Pt<2, T> s, ds;
      unpack<2, T>(X[j], s);
      Stress<2, T> st;
      stress<2, T>(p, s.E, st);
      T sl[2];
      source_slope<2, P, T>(tb, q, geo, m, p, ec, sl);
      const T wq = tb.qw[q] * geo.detJ;
      T o[10];
      if constexpr (TAN) {
        unpack<2, T>(dX[j], ds);
        e2_vol_tan<T>(p, geo, wq, s, st, ds, sl, o);
      } else {
        e2_vol<T>(p, geo, wq, s, st, sl, o);
      }
      T* dst = sI + (size_t)q * 10 * EB + lane;
#pragma unroll
      for (int k = 0; k < 10; ++k) dst[k * EB] = o[k];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();

  // -------------------------------------------------- stage 4: volume contraction, mass terms, rows
  const T* arg = TAN ? x : W;  // the coefficients the mass terms and unused rows take
#pragma unroll
  for (int s = 0; s < C::GS; ++s) {
    const int f = w + s * NW;
    if (f >= S::NF) break;
    e2_contract_volume<P, T>(tb, sI, lane, f, geo, acc[s]);
    if (!live) continue;
    const unsigned eu = (unsigned)e;
#pragma unroll
    for (int i = 0; i < S::NP; ++i) {
      const int row = f * S::NP + i;
      T v = acc[s][i];
      if constexpr (!TAN) {
        if (f < 3) v -= rowld(bold, row, n, eu);
      }
      // unused modes of a lower-order field (wave-uniform test): the row is
      // the coefficient itself
      if (row_unused<2, T>(m, f, i)) v = rowld(arg, row, n, eu);
      rowref(out, row, n, eu) = v;
    }
  }
}

// Diagonal block dR_e/dW_e of a triangle from pointwise tangents.  The
// residual's dependence on the element's own coefficient (g, j) enters only
// through the point states, as phi_j(q) e_g at a volume point and
// phi_j(p) e_g on the element's side of a face point (the neighbour's side
// fixed; at a boundary face the exterior state follows the interior one
// through its own tangent).  The integrands' tangents are linear in that
// direction, so
//   B[(f,i),(g,j)] = sum_q C_fi(o_q^g) phi_j(q) + sum_p L_fi(o_p^g) phi_j(p)
//                    + mass terms,
// where o_q^g (o_p^g) are the volume (face) integrands' tangents along the
// unit direction e_g at the point, and C_fi, L_fi the contraction and lift of
// row (f, i) (the same maps as the element pass's stages 2 and 4).  One
// workgroup per element: phase A, one lane per (point, direction), 24 x 7
// lanes at P3, parks the tangents in LDS; phase B, one lane per (row, column
// field), contracts them with the test functions and writes the row's 10
// entries of that column field.  Against one lane per column evaluating
// every point's tangent along that column (70 evaluations of the stress
// tangent per point at P3), the pointwise work falls by N_p and the
// contraction is a product with the basis tables.
//
// FULL = false assembles only what the block-Jacobi factors read, in their
// compact per-element layout (Schur<2, P>::CB numbers): the depth-velocity
// block A_VV, the velocity rows' stress columns A_UE, the stress rows'
// velocity columns A_EU, and the diagonal of A_EE.  The stress equations'
// integrands do not involve E (their tangents along a stress direction are
// exact zeros, boundaries included), so A_EE is the mass term alone, |J| on
// the diagonal (1 on unused modes), and is written directly; A_hE and A_Eh
// vanish.  25 N_p (row, column field) items instead of 7 N_p * 7: one round
// of 256 lanes at P3, the same values as the whole blocks.
template <int P>
struct JB2 {
  using S = Shape<2, P>;
  static constexpr int NFP = S::NFC * S::NFQ;     // face points
  static constexpr int NPT = S::NQ + NFP;         // points
  static constexpr int NA = NPT * S::NF;          // phase-A items
  static constexpr int NBI = S::BS * S::NF;       // phase-B items (row, column field)
  static constexpr int NT = 256;
};

template <int P, class T, bool FULL>
__device__ __forceinline__ void jac_blocks_tri(const T* __restrict__ W, const T* __restrict__ trW,
                                               T* __restrict__ blocks, const MeshView<T>& m, const DevParams<T>& p,
                                               int e) {
  using S = Shape<2, P>;
  using J = JB2<P>;
  const Tab<2, P, T>& tb = tab<2, P, T>();
  const int n = m.n_el;
  const int t = (int)threadIdx.x;
  __shared__ T sc[S::BS];                      // the element's coefficients
  __shared__ T sv[S::NQ][S::NF][10];           // volume integrand tangents
  __shared__ T sf[J::NFP][S::NF][5];           // face integrand tangents
  __shared__ T snv[S::NFC][2];                 // face normals
  // the reference tables the lanes read at lane-dependent indices
  __shared__ T sphi[S::NQ][S::NP], sdphi[S::NQ][S::NP][2], sfphi[S::NFC][S::NFQ][S::NP];
  for (int k = t; k < S::BS; k += J::NT) sc[k] = W[(size_t)k * n + e];
  if (t < S::NFC * 2) snv[t / 2][t % 2] = m.nrm[(size_t)t * n + e];
  for (int k = t; k < S::NQ * S::NP; k += J::NT) {
    const int q = k / S::NP, i = k % S::NP;
    sphi[q][i] = tb.phi[q][i];
    sdphi[q][i][0] = tb.dphi[q][i][0];
    sdphi[q][i][1] = tb.dphi[q][i][1];
  }
  for (int k = t; k < S::NFC * S::NFQ * S::NP; k += J::NT) {
    const int fc = k / (S::NFQ * S::NP), rr = (k / S::NP) % S::NFQ, i = k % S::NP;
    sfphi[fc][rr][i] = tb.fphi[fc][rr][i];
  }
  __syncthreads();
  Geo<2, T> geo;
  load_geo<2, T>(m, e, geo);
  // ---------------- phase A: pointwise tangents along e_g
  for (int a = t; a < J::NA; a += J::NT) {
    const int pt = a / S::NF, g = a % S::NF;
    T X[S::NF], dX[S::NF];
#pragma unroll
    for (int f = 0; f < S::NF; ++f) dX[f] = f == g ? T(1) : T(0);
    if (pt < S::NQ) {
      const int q = pt;
#pragma unroll
      for (int f = 0; f < S::NF; ++f) {
        T v = T(0);
#pragma unroll
        for (int i = 0; i < S::NP; ++i) v += sphi[q][i] * sc[f * S::NP + i];
        X[f] = v;
      }
      Pt<2, T> st, ds;
      unpack<2, T>(X, st);
      unpack<2, T>(dX, ds);
      Stress<2, T> sg;
      stress<2, T>(p, st.E, sg);
      T sl[2];
      source_slope<2, P, T>(tb, q, geo, m, p, e, sl);
      T o[10];
      e2_vol_tan<T>(p, geo, tb.qw[q] * geo.detJ, st, sg, ds, sl, o);
#pragma unroll
      for (int k = 0; k < 10; ++k) sv[q][g][k] = o[k];
    } else {
      const int kp = pt - S::NQ, fc = kp / S::NFQ, rr = kp % S::NFQ;
      const int code = m.nbr[(size_t)fc * n + e];
#pragma unroll
      for (int f = 0; f < S::NF; ++f) {
        T v = T(0);
#pragma unroll
        for (int i = 0; i < S::NP; ++i) v += sfphi[fc][rr][i] * sc[f * S::NP + i];
        X[f] = v;
      }
      const T nv[2] = {snv[fc][0], snv[fc][1]};
      Pt<2, T> sm, sp, dsm, dsp;
      unpack<2, T>(X, sm);
      unpack<2, T>(dX, dsm);
      if (code >= 0) {
        T Xp[S::NF], z[S::NF];
        load_trace<2, P, T>(trW, n, code >> 2, code & 3, S::NFQ - 1 - rr, Xp);
#pragma unroll
        for (int f = 0; f < S::NF; ++f) z[f] = T(0);
        unpack<2, T>(Xp, sp);
        unpack<2, T>(z, dsp);
      } else {
        exterior<2, T>(p, nv, -1 - code, sm, sp);
        exterior_tan<2, T>(p, nv, -1 - code, dsm, dsp);
      }
      T o[5];
      e2_face_tan<T>(p, nv, tb.fw[rr] * m.hlen[(size_t)fc * n + e], sm, sp, dsm, dsp, o);
#pragma unroll
      for (int k = 0; k < 5; ++k) sf[kp][g][k] = o[k];
    }
  }
  __syncthreads();
  // ---------------- phase B: rows (f, i) of column field g
  using Z = Schur<2, P>;
  T* blk = blocks + (size_t)e * (FULL ? S::BS * S::BS : Z::CB);
  constexpr int NP = S::NP;
  for (int b = t; b < (FULL ? J::NBI : 25 * NP); b += J::NT) {
    int row, g;
    if constexpr (FULL) {
      row = b / S::NF;
      g = b % S::NF;
    } else if (b < 9 * NP) {  // A_VV
      row = b / 3;
      g = b % 3;
    } else if (b < 17 * NP) {  // A_UE
      row = NP + (b - 9 * NP) / 4;
      g = 3 + (b - 9 * NP) % 4;
    } else {  // A_EU
      row = 3 * NP + (b - 17 * NP) / 2;
      g = 1 + (b - 17 * NP) % 2;
    }
    const int f = row / S::NP, i = row % S::NP;
    T out[S::NP];
    if (row_unused<2, T>(m, f, i)) {
#pragma unroll
      for (int j = 0; j < S::NP; ++j) out[j] = (g * S::NP + j == row) ? T(1) : T(0);
    } else {
#pragma unroll
      for (int j = 0; j < S::NP; ++j) out[j] = T(0);
      // volume: C_fi(o_q^g) per point, then times phi_j(q)
      // (for a gradient row (b, a): column a of the metric, selected here so
      // that the geometry is not indexed at run time, which would put it in
      // scratch memory)
      const int bb = f >= 3 ? (f - 3) >> 1 : 0, aa = f >= 3 ? (f - 3) & 1 : 0;
      const T xa0 = aa == 0 ? geo.xi[0][0] : geo.xi[0][1];
      const T xa1 = aa == 0 ? geo.xi[1][0] : geo.xi[1][1];
#pragma unroll 1
      for (int q = 0; q < S::NQ; ++q) {
        const T* o = sv[q][g];
        T c;
        if (f < 3) {
          c = sdphi[q][i][0] * o[2 + f] + sdphi[q][i][1] * o[5 + f];
          if (f > 0) c += sphi[q][i] * o[f - 1];
        } else {
          c = (sdphi[q][i][0] * xa0 + sdphi[q][i][1] * xa1) * o[8 + bb];
        }
#pragma unroll
        for (int j = 0; j < S::NP; ++j) out[j] += c * tb.phi[q][j];
      }
      // faces: L_fi(o_p^g) per point, then times the face basis
#pragma unroll 1
      for (int kp = 0; kp < J::NFP; ++kp) {
        const int fc = kp / S::NFQ, rr = kp % S::NFQ;
        const T* o = sf[kp][g];
        T c;
        if (f < 3) {
          c = o[f];
        } else {
          c = o[3 + bb] * snv[fc][aa];
        }
        c *= sfphi[fc][rr][i];
#pragma unroll
        for (int j = 0; j < S::NP; ++j) out[j] += c * tb.fphi[fc][rr][j];
      }
      // mass terms: |J| / dt on the depth rows, |J| on the gradient rows
      if (g == f && (f == 0 || f >= 3)) {
        const T ms = f == 0 ? geo.detJ * p.inv_dt : geo.detJ;
#pragma unroll
        for (int j = 0; j < S::NP; ++j)
          if (j == i) out[j] += ms;
      }
      // columns of unused modes are unit columns
#pragma unroll
      for (int j = 0; j < S::NP; ++j)
        if (row_unused<2, T>(m, g, j)) out[j] = T(0);
    }
    T* dst;
    if constexpr (FULL) dst = blk + (size_t)row * S::BS + g * NP;
    else if (row < Z::NV && g < 3) dst = blk + row * Z::NV + g * NP;
    else if (row < Z::NV) dst = blk + Z::CUE + (row - NP) * Z::NE + (g - 3) * NP;
    else dst = blk + Z::CEU + (row - Z::NV) * Z::NU + (g - 1) * NP;
#pragma unroll
    for (int j = 0; j < S::NP; ++j) dst[j] = out[j];
  }
  if constexpr (!FULL) {
    // the diagonal of A_EE
    for (int k = t; k < 4 * NP; k += J::NT) {
      const int f = 3 + k / NP, i = k % NP;
      blk[Z::CDG + k] = row_unused<2, T>(m, f, i) ? T(1) : geo.detJ;
    }
  }
}

template <int P, class T, bool FULL>
__global__ void __launch_bounds__(256) k_jac_blocks_tri(const T* __restrict__ W, const T* __restrict__ trW,
                                                         T* __restrict__ blocks, MeshView<T> m, DevParams<T> p) {
  jac_blocks_tri<P, T, FULL>(W, trW, blocks, m, p, xcd_tile(blockIdx.x, gridDim.x));
}

// Element-pass tile shapes (the autotuner's variants v = 0, 1, 2).  On
// triangles a workgroup of 4 waves on a tile of 64 elements, compiled for at
// least 1, 2 or 3 resident waves per SIMD (a register budget of 512, 256 or
// 168 per lane: fewer spills against more latency hiding); the arithmetic is
// the same code in all three, so they give the same bits.  In 1-D the blocked
// kernel with workgroups of 128, 256 or 512 lanes.
template <int D, int V>
constexpr int etile_nt() {
  if constexpr (D == 2) return 256;
  else return kTileNT[V];
}
template <int D, int P, class T, int V>
constexpr int etile_minw() {
  if constexpr (D == 2) return V + 1;
  else return elem_waves<D, P, T>();
}
template <int D, int P, int V>
constexpr int etile_eb() {
  if constexpr (D == 2) return 64;
  else return Blk<D, P, kTileNT[V]>::EB;
}

template <int D, int P, class T, int MODE, int V>
__device__ __forceinline__ void elem_tile(const T* __restrict__ W, const T* __restrict__ x,
                                          const T* __restrict__ bold, T* __restrict__ out,
                                          const T* __restrict__ trW, const MeshView<T>& m, const DevParams<T>& p,
                                          int e0) {
  if constexpr (D == 2) elem2_tile<P, T, MODE, 4>(W, x, bold, out, trW, m, p, e0);
  else elem_blocked_tile<D, P, T, MODE, kTileNT[V]>(W, x, bold, out, trW, m, p, e0);
}

// single-discretisation element pass (variant V)
template <int D, int P, class T, int MODE, int V>
__global__ void __launch_bounds__((etile_nt<D, V>()), (etile_minw<D, P, T, V>()))
    k_elem(const T* __restrict__ W, const T* __restrict__ x, const T* __restrict__ bold, T* __restrict__ out,
           const T* __restrict__ trW, MeshView<T> m, DevParams<T> p) {
  elem_tile<D, P, T, MODE, V>(W, x, bold, out, trW, m, p, xcd_tile(blockIdx.x, gridDim.x) * etile_eb<D, P, V>());
}

}  // namespace bsw
