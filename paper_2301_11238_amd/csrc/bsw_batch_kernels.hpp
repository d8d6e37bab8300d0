// Multi-instance ("batched") kernels: one launch covers every instance of a
// batch that takes part in a stage.  Instances differ in mesh, size,
// parameters and time step but share dimension, order and precision.
//
// A launch receives a BatchSet by value (kernel argument, read through the
// scalar unit): the participating instances in engine-slot order and the
// prefix sum of their tile counts.  A workgroup finds its instance with a
// uniform binary search over that prefix, so tiles never straddle instances
// and nothing a workgroup computes depends on which other instances share the
// launch.  Reductions are per instance with a tile decomposition that depends
// only on the instance's own length: results are bitwise the same whether an
// instance runs alone or in a mix.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bsw_elem2.hpp"

namespace bsw {

constexpr int kMaxBatch = 128;  // instances per batch
constexpr int kVT = 512;        // reals per vector tile (256 lanes x 2)
// FP64 scalars per instance (device array and a host-mapped mirror):
// Gram-Schmidt coefficient rows of even and odd Arnoldi steps, the scales of
// the stored Krylov vectors, the Krylov combination weights and norms, and
// the second Gram-Schmidt pass's weights of the stored vectors.
constexpr int kScStride = 592;
constexpr int kScA = 0, kScB = 72, kScA1 = 144, kScB1 = 216;
constexpr int kScS = 288, kScY = 360, kScN = 432, kScC = 448, kScD = 520;
constexpr int kSlotJ = 1 << 16;  // slot flag: add the instance's Krylov index

// The launch set every batched kernel takes by value (about 1 KB of kernel
// argument; a probe of six kernels per step measured about 0.6 us per KB
// per launch).
struct BatchSet {
  int n;                       // participating instances
  int tile0[kMaxBatch + 1];    // prefix of their tile counts
  uint16_t inst[kMaxBatch];    // engine slot
  uint8_t rows[kMaxBatch];     // per-instance row count (reductions, combinations)
  uint8_t jv[kMaxBatch];       // per-instance Krylov index
};
// the launch set with a per-instance scalar (kb_lin, kb_combine)
struct BatchSetS : BatchSet {
  double s[kMaxBatch];
};

__device__ __forceinline__ int bset_find(const BatchSet& A, int b) {
  int lo = 0, hi = A.n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (A.tile0[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

template <class T>
struct InstDesc {
  MeshView<T> m;
  DevParams<T> p;   // parameters of the current step (1/dt included)
  T* ws;            // state vectors: slot k starts at ws + k * ld
  int64_t ld;
  int64_t len;      // n_f N_p n_el
  int64_t len_v;    // (1 + D) N_p n_el: the entries of the first 1 + D fields
  float* blk;       // block-Jacobi factors (FP32), [number][n_el]
  T* blk_raw;       // diagonal blocks, [n_el][row][col]
  T* trL;           // face traces of the linearisation state
  double* part;     // reduction partials, [row][tile]
  int ntile;        // vector tiles: ceil(len / kVT)
  int ntile_e;      // element tiles of 256: ceil(n_el / 256)
};

template <class T>
__device__ __forceinline__ T* bslot(const InstDesc<T>& I, int s, int j) {
  return I.ws + (int64_t)((s & 0xffff) + ((s & kSlotJ) ? j : 0)) * I.ld;
}

// the device library's wave reductions of doubles (its 32-bit reductions are
// declared by the HIP headers)
extern "C" __device__ __attribute__((const)) double __ockl_wfred_add_f64(double);
extern "C" __device__ __attribute__((const)) double __ockl_wfred_max_f64(double);
extern "C" __device__ __attribute__((const)) double __ockl_wfred_min_f64(double);

// 256-lane sum / max / min (a wave reduction per wave, then the four wave
// results in wave order: a fixed order); the result is valid on every lane.
// Called by all 256 threads with every lane active.
__device__ __forceinline__ double bred(double v, int op) {
  __shared__ double sh[4];
  const double w = op == 0 ? __ockl_wfred_add_f64(v) : (op == 1 ? __ockl_wfred_max_f64(v) : __ockl_wfred_min_f64(v));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int k = 1; k < 4; ++k) r = op == 0 ? r + sh[k] : (op == 1 ? fmax(r, sh[k]) : fmin(r, sh[k]));
  __syncthreads();
  return r;
}

// Sum (op 0), maximum (1) or minimum (2) of the partials p[0 .. nt) by a
// 256-lane workgroup, in a fixed order: lane l keeps eight accumulators,
// accumulator u taking p[2048 k + 256 u + l] for k = 0, 1, ...; the eight are
// combined in order u = 0..7, then over the workgroup (bred).  The eight loads
// of a round are independent, so a round costs one memory latency, not eight.
// Every fold of one set of partials goes through here, so the result does
// not depend on which kernel folded it.
__device__ __forceinline__ double fold_partials(const double* __restrict__ p, int nt, int op) {
  const double init = op == 0 ? 0.0 : (op == 1 ? -INFINITY : INFINITY);
  double a[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) a[u] = init;
  for (int base = (int)threadIdx.x; base < nt; base += 2048) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = base + 256 * u < nt ? p[base + 256 * u] : init;
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = op == 0 ? a[u] + v[u] : (op == 1 ? fmax(a[u], v[u]) : fmin(a[u], v[u]));
  }
  double acc = a[0];
#pragma unroll
  for (int u = 1; u < 8; ++u) acc = op == 0 ? acc + a[u] : (op == 1 ? fmax(acc, a[u]) : fmin(acc, a[u]));
  return bred(acc, op);
}

// ------------------------------------------------------------------ element stages
template <int D, int P, class T>
__global__ void __launch_bounds__(256) kb_step_begin(const InstDesc<T>* __restrict__ ds, BatchSet A, int sW,
                                                      int sB) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int e = (blockIdx.x - A.tile0[ai]) * 256 + threadIdx.x;
  if (e < I.m.n_el) step_begin_elem<D, P, T>(bslot(I, sW, 0), bslot(I, sB, 0), I.m, I.p, e);
}

// face traces of slot sX (the linearisation state) into trL; tiles of 256
// (field, face, element) items
template <int D, int P, class T>
__global__ void __launch_bounds__(256) kb_trace(const InstDesc<T>* __restrict__ ds, BatchSet A, int sX) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int64_t item = (int64_t)(blockIdx.x - A.tile0[ai]) * 256 + threadIdx.x;
  if (item < (int64_t)Shape<D, P>::NF * Shape<D, P>::NFC * I.m.n_el)
    trace_item<D, P, T>(bslot(I, sX, A.jv[ai]), I.trL, I.m.n_el, item);
}

// MODE 0: R = residual(W; b_old); MODE 1: y = J(W) x with the traces of W in
// trL (the neighbours' side of the pass's argument, W or x, is evaluated in
// the pass from their coefficients)
// V: the element-tile shape (elem_tile's variant), chosen by the autotuner
template <int D, int P, class T, int MODE, int V>
__global__ void __launch_bounds__((etile_nt<D, V>()), (etile_minw<D, P, T, V>())) kb_elem(const InstDesc<T>* __restrict__ ds, BatchSet A, int sW, int sX,
                                                     int sB, int sOut) {
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int ai = bset_find(A, b);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int j = A.jv[ai];
  const int e0 = (b - A.tile0[ai]) * etile_eb<D, P, V>();
  elem_tile<D, P, T, MODE, V>(bslot(I, sW, j), MODE == 1 ? bslot(I, sX, j) : nullptr,
                              MODE == 0 ? bslot(I, sB, j) : nullptr, bslot(I, sOut, j),
                              MODE == 0 ? nullptr : I.trL, I.m, I.p, e0);
}

template <int D, int P, class T>
__global__ void __launch_bounds__(256) kb_jac_columns(const InstDesc<T>* __restrict__ ds, BatchSet A, int sW) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  jac_columns_elem<D, P, T>(bslot(I, sW, 0), I.trL, I.blk_raw, I.m, I.p, blockIdx.x - A.tile0[ai]);
}

// the parts of the diagonal blocks of triangles the block-Jacobi factors
// read, one element per workgroup (k_jac_blocks_tri)
template <int P, class T>
__global__ void __launch_bounds__(256) kb_jac_blocks_tri(const InstDesc<T>* __restrict__ ds, BatchSet A, int sW) {
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int ai = bset_find(A, b);
  const InstDesc<T> I = ds[A.inst[ai]];
  jac_blocks_tri<P, T, false>(bslot(I, sW, 0), I.trL, I.blk_raw, I.m, I.p, b - A.tile0[ai]);
}

// a pointer the whole wave holds, moved to scalar registers (so that the
// compiler treats loads through it at uniform offsets as scalar loads)
template <class Q>
__device__ __forceinline__ Q* wave_uniform(Q* q) {
  const uint64_t u = (uint64_t)(uintptr_t)q;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return (Q*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

// block-Jacobi factors, four elements per workgroup (k_schur_build)
template <int D, int P, class T>
__global__ void __launch_bounds__(256) kb_schur_build(const InstDesc<T>* __restrict__ ds, BatchSet A) {
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int ai = bset_find(A, b);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int n = __builtin_amdgcn_readfirstlane(I.m.n_el);
  // (the instance search runs in vector registers: the element index is
  // made wave-uniform explicitly)
  const int e = __builtin_amdgcn_readfirstlane((b - A.tile0[ai]) * kSchurEPB + ((int)threadIdx.x >> 6));
  schur_build_elem<D, P, T>(wave_uniform(I.blk_raw), wave_uniform(I.blk), n, e, e < n);
}

// y = M^{-1} x on Krylov slot j, 64 elements per workgroup (k_schur_apply)
template <int D, int P, class T>
__global__ void __launch_bounds__(256) kb_prec_apply(const InstDesc<T>* __restrict__ ds, BatchSet A, int sX,
                                                      int sY) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int j = A.jv[ai];
  schur_apply_tile<D, P, T>(I.blk, bslot(I, sX, j), bslot(I, sY, j), I.m, I.p.bc,
                            ((int)blockIdx.x - A.tile0[ai]) * kPrecEB, [] { return 1.0; });
}

// mass, active area, max wave speed, min depth per 256-element tile
template <int D, int P, class T>
__global__ void __launch_bounds__(256) kb_diag(const InstDesc<T>* __restrict__ ds, BatchSet A, int sW) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int t = blockIdx.x - A.tile0[ai];
  const int e = t * 256 + threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, INFINITY};
  if (e < I.m.n_el)
    diag_elem<D, P, T>(bslot(I, sW, 0), I.m, (double)I.p.g, (double)I.p.s0 / (double)I.p.gam, e, v);
  const int ops[4] = {0, 0, 1, 2};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double x = bred(v[r], ops[r]);
    if (threadIdx.x == 0) I.part[(int64_t)r * I.ntile_e + t] = x;
  }
}

// ------------------------------------------------------------------ vector stages (tiles of kVT reals)
// y = a x + b z; flag 1: a = per-instance scalar, 2: b = per-instance scalar,
// 4: y = 0, 8: no z term
template <class T>
__global__ void __launch_bounds__(256) kb_lin(const InstDesc<T>* __restrict__ ds, BatchSetS A, int sy, int sx, int sz,
                                               double ca, double cb, int flags) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int j = A.jv[ai];
  const double a = (flags & 1) ? A.s[ai] : ca, b = (flags & 2) ? A.s[ai] : cb;
  T* y = bslot(I, sy, j);
  const T* x = bslot(I, sx, j);
  const T* z = bslot(I, sz, j);
  const int64_t i0 = (int64_t)(blockIdx.x - A.tile0[ai]) * kVT + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kVT / 256; ++k) {
    const int64_t i = i0 + k * 256;
    if (i >= I.len) break;
    if (flags & 4) y[i] = T(0);
    else if (flags & 8) y[i] = (T)(a * (double)x[i]);
    else y[i] = (T)(a * (double)x[i] + b * (double)z[i]);
  }
}

// y = s (w - sum_{i < rows} c_i V_i) with c in the instance's scalar row
// `coff`; flag 1: s = per-instance scalar (else 1), 2: no w term (y = sum),
// 4: y += (instead of =) the combination, with sign sgn, 8: c_i sigma_i
template <class T>
__global__ void __launch_bounds__(256) kb_combine(const InstDesc<T>* __restrict__ ds, BatchSetS A, const double* sc,
                                                   int coff, int sV0, int sw, int sy, double sgn, int flags) {
  const int ai = bset_find(A, blockIdx.x);
  const int slot = A.inst[ai];
  const InstDesc<T> I = ds[slot];
  const int j = A.jv[ai];
  const int rows = A.rows[ai];
  const double s = (flags & 1) ? A.s[ai] : 1.0;
  const double* c = sc + (int64_t)slot * kScStride + coff;
  const double* sg = sc + (int64_t)slot * kScStride + kScS;
  const T* V = bslot(I, sV0, j);
  const T* w = bslot(I, sw, j);
  T* y = bslot(I, sy, j);
  const int64_t i0 = (int64_t)(blockIdx.x - A.tile0[ai]) * kVT + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kVT / 256; ++k) {
    const int64_t i = i0 + k * 256;
    if (i >= I.len) break;
    double acc = 0.0;
    if (flags & 8)
      for (int r = 0; r < rows; ++r) acc += c[r] * sg[r] * (double)V[(int64_t)r * I.ld + i];
    else
      for (int r = 0; r < rows; ++r) acc += c[r] * (double)V[(int64_t)r * I.ld + i];
    if (flags & 4) y[i] = (T)((double)y[i] + sgn * acc);
    else if (flags & 2) y[i] = (T)(s * acc);
    else y[i] = (T)(s * ((double)w[i] - acc));
  }
}

// ------------------------------------------------------------------ Krylov (Arnoldi) stages
// The Krylov vectors are stored unnormalised: V_true[r] = sigma_r V[r] with
// sigma_r = sc[kScS + r], so each new vector's norm is computed exactly from
// the vector itself and no pass only rescales.
//
// Gram-Schmidt with delayed reorthogonalisation (the DCGS2 scheme of
// Swirydowicz, Langou, Ananthan, Yang and Thomas, 2020): at Arnoldi step j
// the basis v_0..v_{j-1} is final, y_j = sigma_j V[j] is the new direction
// after one projection (unit norm, not yet reorthogonalised) and w = A M^-1
// y_j.  One pass over the basis forms s = V^T y_j, a = y_j . y_j,
// t = V^T w and b = y_j . w; a second pass writes the reorthogonalised
// v_j = (y_j - V s) / rho, rho = sqrt(a - s . s), and the next direction
// u_{j+1} = (w - V t - c v_j) / rho, c = v_j . w = (b - s . t) / rho, which
// is w's projection out of the final basis scaled as A M^-1 v_j would be.
// The Hessenberg column of step j-1 is completed on the host from s and
// rho (its Arnoldi relation took u_j, not v_j).  Two reads of the basis per
// step instead of the three of classical Gram-Schmidt with a second pass.

// red[u][tid] holds the 256 products of rows r0 + u (u < 8) of one tile:
// wave w sums rows 2w and 2w + 1, each lane four consecutive products, then
// one wave reduction (a fixed order); the row sums below nrow go to the
// tile's partials.  Called by all 256 threads, between barriers.
__device__ __forceinline__ void fold_group(const double (&red)[8][257], int r0, int nrow, double* __restrict__ part,
                                           int ntile, int t) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int u = 2 * wv + h;
    double s = red[u][lane * 4];
#pragma unroll
    for (int m = 1; m < 4; ++m) s += red[u][lane * 4 + m];
    s = __ockl_wfred_add_f64(s);
    if (lane == 0 && r0 + u < nrow) part[(int64_t)(r0 + u) * ntile + t] = s;
  }
}

// Gram-Schmidt pass 1 of step j: per-tile partials of the rows
// 2r = V[r] . V[j] and 2r + 1 = V[r] . w for r <= j (the last pair gives
// y_j . y_j and y_j . w once scaled), eight partial rows (four basis rows)
// per round: products transposed through LDS and summed per row by
// fold_group (a fixed order).
template <class T>
__global__ void __launch_bounds__(256) kb_gs_dots(const InstDesc<T>* __restrict__ ds, BatchSet A, int sV0, int sw) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int t = blockIdx.x - A.tile0[ai];
  const int nv = A.jv[ai] + 1, rows = 2 * nv;
  const T* V = bslot(I, sV0, 0);
  const T* w = bslot(I, sw, 0);
  const T* y = V + (int64_t)(nv - 1) * I.ld;
  const int64_t i0 = (int64_t)t * kVT + threadIdx.x, i1 = i0 + 256;
  const bool in0 = i0 < I.len, in1 = i1 < I.len;
  const double y0 = in0 ? (double)y[i0] : 0.0, y1 = in1 ? (double)y[i1] : 0.0;
  const double w0 = in0 ? (double)w[i0] : 0.0, w1 = in1 ? (double)w[i1] : 0.0;
  __shared__ double red[8][257];
  const int tid = threadIdx.x;
  for (int r0 = 0; r0 < rows; r0 += 8) {
#pragma unroll
    for (int u = 0; u < 8; u += 2) {
      const int r = (r0 + u) >> 1;
      double a = 0.0, c = 0.0;
      if (r < nv) {
        const T* v = V + (int64_t)r * I.ld;
        const double x0 = in0 ? (double)v[i0] : 0.0, x1 = in1 ? (double)v[i1] : 0.0;
        a = x0 * y0 + x1 * y1;
        c = x0 * w0 + x1 * w1;
      }
      red[u][tid] = a;
      red[u + 1][tid] = c;
    }
    __syncthreads();
    fold_group(red, r0, rows, I.part, I.ntile, t);
    __syncthreads();
  }
}

// kb_gs_dots for instances with j + 1 <= kRowsCached: every lane first loads
// its entries of V_0..V_j (all loads in flight at once, not four rows per
// round trip); the rows are then reduced as in kb_gs_dots, in the same order
constexpr int kRowsCached = 32;

template <class T>
__global__ void __launch_bounds__(256) kb_gs_dots_cached(const InstDesc<T>* __restrict__ ds, BatchSet A, int sV0,
                                                          int sw) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int t = blockIdx.x - A.tile0[ai];
  const int nv = A.jv[ai] + 1, rows = 2 * nv;
  const T* V = bslot(I, sV0, 0);
  const T* w = bslot(I, sw, 0);
  const T* y = V + (int64_t)(nv - 1) * I.ld;
  const int64_t i0 = (int64_t)t * kVT + threadIdx.x, i1 = i0 + 256;
  const bool in0 = i0 < I.len, in1 = i1 < I.len;
  T v0[kRowsCached], v1[kRowsCached];
#pragma unroll
  for (int r = 0; r < kRowsCached; ++r) {
    const T* v = V + (int64_t)r * I.ld;
    v0[r] = r < nv && in0 ? v[i0] : T(0);
    v1[r] = r < nv && in1 ? v[i1] : T(0);
  }
  const double y0 = in0 ? (double)y[i0] : 0.0, y1 = in1 ? (double)y[i1] : 0.0;
  const double w0 = in0 ? (double)w[i0] : 0.0, w1 = in1 ? (double)w[i1] : 0.0;
  __shared__ double red[8][257];
  const int tid = threadIdx.x;
#pragma unroll
  for (int r0 = 0; r0 < 2 * kRowsCached; r0 += 8) {
    if (r0 < rows) {
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        const int r = (r0 + u) >> 1;
        const double x0 = (double)v0[r], x1 = (double)v1[r];
        red[u][tid] = x0 * y0 + x1 * y1;
        red[u + 1][tid] = x0 * w0 + x1 * w1;
      }
      __syncthreads();
      fold_group(red, r0, rows, I.part, I.ntile, t);
      __syncthreads();
    }
  }
}

// rho and c of step j from the folded rows s_r = sA[r] (r < j), a = sA[j],
// t_r = sB[r], b = sB[j]; at j = 0, y_0 is the normalised residual itself
// (rho = 1).  Every caller evaluates them in this order.
__device__ __forceinline__ void gs_rho_c(const double* __restrict__ sA, const double* __restrict__ sB, int j,
                                         double& rho, double& c) {
  if (j == 0) {
    rho = 1.0;
    c = sB[0];
    return;
  }
  double ss = 0.0, st = 0.0;
  for (int r = 0; r < j; ++r) {
    ss += sA[r] * sA[r];
    st += sA[r] * sB[r];
  }
  const double d = sA[j] - ss;
  rho = d > 0.0 ? sqrt(d) : 0.0;
  c = rho > 0.0 ? (sB[j] - st) / rho : 0.0;
}

// Gram-Schmidt pass 2 of step j (coefficients in rows offA, offB of the
// instance's scalars, the weights of the V[r] at kScC, kScD): V[j] <- (V[j]
// - sum_{r<j} (s_r sigma_r / sigma_j) V[r]) / rho, so that sigma_j V[j] is
// v_j; V[j+1] <- (w - sum_{r<j} t_r sigma_r V[r] - c v_j) / rho,
// unnormalised, with the partials of its squared norm.  The instance's first
// workgroup stores rho and c (rows offR, offC) in sc and its host mirror
// sch.  The basis is read sixteen rows per round (150 registers, three
// waves per SIMD: 279 us per call at C3 against 296 us with every row's
// loads issued at once at two waves per SIMD).
template <class T>
__global__ void __launch_bounds__(256) kb_gs_update(const InstDesc<T>* __restrict__ ds, BatchSet A,
                                                     double* __restrict__ sc, double* __restrict__ sch, int offA,
                                                     int offB, int offR, int offC, int sV0, int sw) {
  constexpr int G = 16;
  const int ai = bset_find(A, blockIdx.x);
  const int slot = __builtin_amdgcn_readfirstlane(A.inst[ai]);
  const InstDesc<T> I = ds[slot];
  const int t = blockIdx.x - A.tile0[ai];
  const int j = __builtin_amdgcn_readfirstlane(A.jv[ai]);
  const double* sd = wave_uniform(sc + (int64_t)slot * kScStride);
  const double* s = sd + offA;
  const double* tt = sd + offB;
  const double* sg = sd + kScS;
  double rho, c;
  gs_rho_c(s, tt, j, rho, c);
  if (t == 0 && threadIdx.x == 0) {
    double* d = sc + (int64_t)slot * kScStride;
    double* h = sch + (int64_t)slot * kScStride;
    d[offR] = rho;
    h[offR] = rho;
    d[offC] = c;
    h[offC] = c;
  }
  const double rinv = rho > 0.0 ? 1.0 / rho : 0.0;
  const double sj = sg[j];
  const double* ws = sd + kScC;  // s_r sigma_r / sigma_j
  const double* wt = sd + kScD;  // t_r sigma_r
  T* V = bslot(I, sV0, 0);
  const T* w = bslot(I, sw, 0);
  T* vj = V + (int64_t)j * I.ld;
  T* un = V + (int64_t)(j + 1) * I.ld;
  const int64_t i0 = (int64_t)t * kVT + threadIdx.x, i1 = i0 + 256;
  const bool in0 = i0 < I.len, in1 = i1 < I.len;
  double p0 = in0 ? (double)vj[i0] : 0.0, p1 = in1 ? (double)vj[i1] : 0.0;
  double a0 = in0 ? (double)w[i0] : 0.0, a1 = in1 ? (double)w[i1] : 0.0;
  for (int r0 = 0; r0 < j; r0 += G) {
    double x0[G], x1[G], cs[G], ct[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int r = r0 + u;
      const bool ok = r < j;
      const int rr = ok ? r : 0;
      const T* v = V + (int64_t)rr * I.ld;
      cs[u] = ok ? ws[rr] : 0.0;
      ct[u] = ok ? wt[rr] : 0.0;
      x0[u] = ok && in0 ? (double)v[i0] : 0.0;
      x1[u] = ok && in1 ? (double)v[i1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      p0 -= cs[u] * x0[u];
      p1 -= cs[u] * x1[u];
      a0 -= ct[u] * x0[u];
      a1 -= ct[u] * x1[u];
    }
  }
  double q = 0.0;
  if (j == 0) {
    // v_0 is final as stored
    if (in0) a0 -= c * sj * p0;
    if (in1) a1 -= c * sj * p1;
  } else {
    if (in0) { const T v = (T)(p0 * rinv); vj[i0] = v; a0 -= c * sj * (double)v; }
    if (in1) { const T v = (T)(p1 * rinv); vj[i1] = v; a1 -= c * sj * (double)v; }
  }
  if (in0) { const T u = (T)(a0 * rinv); un[i0] = u; q += (double)u * (double)u; }
  if (in1) { const T u = (T)(a1 * rinv); un[i1] = u; q += (double)u * (double)u; }
  const double x = bred(q, 0);
  if (threadIdx.x == 0) I.part[t] = x;
}

// z = sigma_j M^{-1} V_j (the preconditioner on the stored Krylov vector j)
// Where A.rows[ai] is set, V_j was written by the previous step's
// kb_gs_update and its squared-norm partials are still in I.part: every
// workgroup folds them (the fold of kb_rows_final, same order) into
// sigma_j = 1 / ||V_j||, after the loads of its first phase have gone out,
// and the instance's first workgroup stores sigma_j and the norm (row offN)
// in sc and its host mirror sch.  Elsewhere sigma_j is read from sc.
template <int D, int P, class T>
__global__ void __launch_bounds__(256) kb_prec_krylov(const InstDesc<T>* __restrict__ ds, BatchSet A,
                                                       double* __restrict__ sc, double* __restrict__ sch, int offN,
                                                       int sV0, int sZ) {
  const int b = blockIdx.x;
  const int ai = bset_find(A, b);
  const int slot = A.inst[ai];
  const InstDesc<T> I = ds[slot];
  const int j = A.jv[ai];
  const bool fold = A.rows[ai] != 0;
  const bool first = b == A.tile0[ai];
  auto sigma = [&]() -> double {
    if (!fold) return sc[(int64_t)slot * kScStride + kScS + j];
    const double nrm = sqrt(fold_partials(I.part, I.ntile, 0));
    const double sgm = nrm > 0.0 ? 1.0 / nrm : 0.0;
    if (first && threadIdx.x == 0) {
      double* sd = sc + (int64_t)slot * kScStride;
      double* sh = sch + (int64_t)slot * kScStride;
      sd[kScS + j] = sgm;
      sh[kScS + j] = sgm;
      sd[offN] = nrm;
      sh[offN] = nrm;
    }
    return sgm;
  };
  schur_apply_tile<D, P, T>(I.blk, bslot(I, sV0, 0) + (int64_t)j * I.ld, bslot(I, sZ, 0), I.m, I.p.bc,
                            (b - A.tile0[ai]) * kPrecEB, sigma);
}

// ------------------------------------------------------------------ per-instance reductions
// partials of sum x^2 (op 0) or max |x| (op 1) over up to two slots
// (vonly: only the first 1 + D fields, e.g. of b_old)
template <class T>
__global__ void __launch_bounds__(256) kb_vred(const InstDesc<T>* __restrict__ ds, BatchSet A, int s0, int s1,
                                                int op, int vonly) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int r = blockIdx.y;
  const int t = blockIdx.x - A.tile0[ai];
  const T* x = bslot(I, r == 0 ? s0 : s1, A.jv[ai]);
  const int64_t lim = vonly ? I.len_v : I.len;
  double acc = 0.0;
  const int64_t i0 = (int64_t)t * kVT + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kVT / 256; ++k) {
    const int64_t i = i0 + k * 256;
    if (i < lim) {
      const double v = (double)x[i];
      acc = op == 0 ? acc + v * v : fmax(acc, fabs(v));
    }
  }
  const double y = bred(acc, op == 0 ? 0 : 1);
  if (threadIdx.x == 0) I.part[(int64_t)r * I.ntile + t] = y;
}

// final pass: one workgroup per (instance, row) folds the instance's partials
// in a fixed order; op of row r is bits 2r..2r+1 of ops (0 sum, 1 max, 2 min)
// scl: rows r <= j are multiplied by sigma_r (dots against stored Krylov
// vectors); sig >= 0: row 0 is a sum of squares, its square root is written
// and sigma_{j + sig} = 1 / root (0 for a zero vector); off2 >= 0: the row
// pairs of kb_gs_dots, row 2r scaled by sigma_r sigma_j to off + r, row
// 2r + 1 by sigma_r to off2 + r, and for r < j the weights kb_gs_update
// gives the stored V[r] (device only): s_r sigma_r / sigma_j at kScC + r,
// t_r sigma_r at kScD + r
template <class T>
__global__ void __launch_bounds__(256) kb_rows_final(const InstDesc<T>* __restrict__ ds, BatchSet A, int etile,
                                                      unsigned ops, double* sc, double* sch, int off, int scl,
                                                      int sig, int off2) {
  const int ai = blockIdx.x;
  const int slot = A.inst[ai];
  const InstDesc<T> I = ds[slot];
  const int r = blockIdx.y;
  if (r >= A.rows[ai]) return;
  const int op = r < 16 ? (int)((ops >> (2 * r)) & 3u) : 0;
  const int nt = etile ? I.ntile_e : I.ntile;
  double x = fold_partials(I.part + (int64_t)r * nt, nt, op);
  if (threadIdx.x == 0) {
    double* s = sc + (int64_t)slot * kScStride;
    double* sh = sch + (int64_t)slot * kScStride;
    const int j = A.jv[ai];
    if (off2 >= 0) {
      const int q = r >> 1;
      const double sq = s[kScS + q];
      x *= sq;
      if (r & 1) {
        s[off2 + q] = x;
        sh[off2 + q] = x;
        if (q < j) s[kScD + q] = x * sq;
      } else {
        const double sj = s[kScS + j];
        x *= sj;
        s[off + q] = x;
        sh[off + q] = x;
        if (q < j) s[kScC + q] = sj > 0.0 ? x * sq * (1.0 / sj) : 0.0;
      }
      return;
    }
    if (sig >= 0) {
      x = sqrt(x);
      const double inv = x > 0.0 ? 1.0 / x : 0.0;
      s[kScS + j + sig] = inv;
      sh[kScS + j + sig] = inv;
    } else if (scl && r <= j) {
      x *= s[kScS + r];
    }
    s[off + r] = x;
    sh[off + r] = x;
  }
}

}  // namespace bsw
