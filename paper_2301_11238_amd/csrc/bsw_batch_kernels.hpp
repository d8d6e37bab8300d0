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

#include "bsw_kernels.hpp"

namespace bsw {

constexpr int kMaxBatch = 128;  // instances per batch
constexpr int kVT = 2048;       // reals per vector tile (256 lanes x 8)
constexpr int kScStride = 144;  // FP64 scalars per instance: two rows of 72
constexpr int kScA = 0, kScB = 72;
constexpr int kSlotJ = 1 << 16;  // slot flag: add the instance's Krylov index

struct BatchSet {
  int n;                       // participating instances
  int tile0[kMaxBatch + 1];    // prefix of their tile counts
  uint16_t inst[kMaxBatch];    // engine slot
  uint8_t rows[kMaxBatch];     // per-instance row count (reductions, combinations)
  uint8_t jv[kMaxBatch];       // per-instance Krylov index
  double s[kMaxBatch];         // per-instance scalar
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
  T* blk;           // block-Jacobi inverses, [row][col][n_el]
  T* blk_raw;       // diagonal blocks, [n_el][row][col]
  T* trL;           // face traces of the linearisation state
  T* trA;           // face traces of the last residual argument
  T* trX;           // face traces of the last Jacobian argument
  double* part;     // reduction partials, [row][tile]
  int ntile;        // vector tiles: ceil(len / kVT)
  int ntile_e;      // element tiles of 256: ceil(n_el / 256)
};

template <class T>
__device__ __forceinline__ T* bslot(const InstDesc<T>& I, int s, int j) {
  return I.ws + (int64_t)((s & 0xffff) + ((s & kSlotJ) ? j : 0)) * I.ld;
}

// 256-lane tree sum / max / min; the result is valid on lane 0
__device__ __forceinline__ double bred(double v, int op) {
  __shared__ double sh[256];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double a = sh[threadIdx.x], b = sh[threadIdx.x + s];
      sh[threadIdx.x] = op == 0 ? a + b : (op == 1 ? fmax(a, b) : fmin(a, b));
    }
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
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

// face traces of slot sX into trL (which 0), trA (1) or trX (2); 256 elements per tile
template <int D, int P, class T>
__global__ void __launch_bounds__(256) kb_trace(const InstDesc<T>* __restrict__ ds, BatchSet A, int sX, int which) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int e = (blockIdx.x - A.tile0[ai]) * 256 + threadIdx.x;
  T* tr = which == 0 ? I.trL : (which == 1 ? I.trA : I.trX);
  if (e < I.m.n_el) trace_elem<D, P, T>(bslot(I, sX, A.jv[ai]), tr, I.m.n_el, e);
}

// MODE 0: R = residual(W; b_old) with the traces in trA; MODE 1: y = J(W) x
// with the traces of W in trL and of x in trX
template <int D, int P, class T, int MODE>
__global__ void __launch_bounds__(256) kb_elem(const InstDesc<T>* __restrict__ ds, BatchSet A, int sW, int sX,
                                                int sB, int sOut) {
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int ai = bset_find(A, b);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int j = A.jv[ai];
  const int e0 = (b - A.tile0[ai]) * Blk<D, P>::EB;
  elem_blocked_tile<D, P, T, MODE>(bslot(I, sW, j), MODE == 1 ? bslot(I, sX, j) : nullptr,
                                   MODE == 0 ? bslot(I, sB, j) : nullptr, bslot(I, sOut, j),
                                   MODE == 0 ? I.trA : I.trL, MODE == 1 ? I.trX : nullptr, I.m, I.p, e0);
}

template <int D, int P, class T>
__global__ void __launch_bounds__(128) kb_jac_columns(const InstDesc<T>* __restrict__ ds, BatchSet A, int sW) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  jac_columns_elem<D, P, T>(bslot(I, sW, 0), I.trL, I.blk_raw, I.m, I.p, blockIdx.x - A.tile0[ai]);
}

template <int BS, class T>
__global__ void __launch_bounds__(64) kb_block_inverse(const InstDesc<T>* __restrict__ ds, BatchSet A) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  block_inverse_elem<BS, T>(I.blk_raw, I.blk, I.m.n_el, blockIdx.x - A.tile0[ai]);
}

template <int BS, class T>
__global__ void __launch_bounds__(256) kb_block_apply(const InstDesc<T>* __restrict__ ds, BatchSet A, int sX,
                                                       int sY) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int j = A.jv[ai];
  const int64_t idx = (int64_t)(blockIdx.x - A.tile0[ai]) * 256 + threadIdx.x;
  if (idx < (int64_t)BS * I.m.n_el) block_apply_item<BS, T>(I.blk, bslot(I, sX, j), bslot(I, sY, j), I.m.n_el, idx);
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
__global__ void __launch_bounds__(256) kb_lin(const InstDesc<T>* __restrict__ ds, BatchSet A, int sy, int sx, int sz,
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
// 4: y += (instead of =) the combination, with sign sgn
template <class T>
__global__ void __launch_bounds__(256) kb_combine(const InstDesc<T>* __restrict__ ds, BatchSet A, const double* sc,
                                                   int coff, int sV0, int sw, int sy, double sgn, int flags) {
  const int ai = bset_find(A, blockIdx.x);
  const int slot = A.inst[ai];
  const InstDesc<T> I = ds[slot];
  const int j = A.jv[ai];
  const int rows = A.rows[ai];
  const double s = (flags & 1) ? A.s[ai] : 1.0;
  const double* c = sc + (int64_t)slot * kScStride + coff;
  const T* V = bslot(I, sV0, j);
  const T* w = bslot(I, sw, j);
  T* y = bslot(I, sy, j);
  const int64_t i0 = (int64_t)(blockIdx.x - A.tile0[ai]) * kVT + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kVT / 256; ++k) {
    const int64_t i = i0 + k * 256;
    if (i >= I.len) break;
    double acc = 0.0;
    for (int r = 0; r < rows; ++r) acc += c[r] * (double)V[(int64_t)r * I.ld + i];
    if (flags & 4) y[i] = (T)((double)y[i] + sgn * acc);
    else if (flags & 2) y[i] = (T)(s * acc);
    else y[i] = (T)(s * ((double)w[i] - acc));
  }
}

// ------------------------------------------------------------------ per-instance reductions
// partials of V_r . w for r < rows (and w . w as the last row when self)
template <class T>
__global__ void __launch_bounds__(256) kb_multidot(const InstDesc<T>* __restrict__ ds, BatchSet A, int sV0, int sw,
                                                    int self) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int rows = A.rows[ai];
  const int r = blockIdx.y;
  if (r >= rows) return;
  const int t = blockIdx.x - A.tile0[ai];
  const T* w = bslot(I, sw, 0);
  const T* v = (self && r == rows - 1) ? w : bslot(I, sV0, 0) + (int64_t)r * I.ld;
  double acc = 0.0;
  const int64_t i0 = (int64_t)t * kVT + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kVT / 256; ++k) {
    const int64_t i = i0 + k * 256;
    if (i < I.len) acc += (double)v[i] * (double)w[i];
  }
  const double x = bred(acc, 0);
  if (threadIdx.x == 0) I.part[(int64_t)r * I.ntile + t] = x;
}

// partials of sum x^2 (op 0) or max |x| (op 1) over up to two slots
template <class T>
__global__ void __launch_bounds__(256) kb_vred(const InstDesc<T>* __restrict__ ds, BatchSet A, int s0, int s1,
                                                int op) {
  const int ai = bset_find(A, blockIdx.x);
  const InstDesc<T> I = ds[A.inst[ai]];
  const int r = blockIdx.y;
  const int t = blockIdx.x - A.tile0[ai];
  const T* x = bslot(I, r == 0 ? s0 : s1, A.jv[ai]);
  double acc = 0.0;
  const int64_t i0 = (int64_t)t * kVT + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kVT / 256; ++k) {
    const int64_t i = i0 + k * 256;
    if (i < I.len) {
      const double v = (double)x[i];
      acc = op == 0 ? acc + v * v : fmax(acc, fabs(v));
    }
  }
  const double y = bred(acc, op == 0 ? 0 : 1);
  if (threadIdx.x == 0) I.part[(int64_t)r * I.ntile + t] = y;
}

// final pass: one workgroup per (instance, row) folds the instance's partials
// in a fixed order; op of row r is bits 2r..2r+1 of ops (0 sum, 1 max, 2 min)
template <class T>
__global__ void __launch_bounds__(256) kb_rows_final(const InstDesc<T>* __restrict__ ds, BatchSet A, int etile,
                                                      unsigned ops, double* sc, double* sch, int off) {
  const int ai = blockIdx.x;
  const int slot = A.inst[ai];
  const InstDesc<T> I = ds[slot];
  const int r = blockIdx.y;
  if (r >= A.rows[ai]) return;
  const int op = r < 16 ? (int)((ops >> (2 * r)) & 3u) : 0;
  const int nt = etile ? I.ntile_e : I.ntile;
  double acc = op == 0 ? 0.0 : (op == 1 ? -INFINITY : INFINITY);
  for (int t = threadIdx.x; t < nt; t += 256) {
    const double v = I.part[(int64_t)r * nt + t];
    acc = op == 0 ? acc + v : (op == 1 ? fmax(acc, v) : fmin(acc, v));
  }
  const double x = bred(acc, op);
  if (threadIdx.x == 0) {
    sc[(int64_t)slot * kScStride + off + r] = x;
    sch[(int64_t)slot * kScStride + off + r] = x;
  }
}

}  // namespace bsw
