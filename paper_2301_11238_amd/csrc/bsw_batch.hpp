// Batched solves and the solve server (host side).  Part of the library's
// single translation unit: included at the end of bsw_lib.hip, it uses the
// handles, dispatch helpers and single-instance entry points defined there.
//
// BatchEngine<T> keeps up to kMaxBatch resident 2-D instances of one order and
// precision and advances all of them by one backward-Euler step per call of
// step_all().  Every stage (b_old, residual, linearisation, block-Jacobi and
// matrix-free Jacobian applies, Krylov vector work, reductions) is one launch
// over the instances that take part in it.  Newton, backtracking and
// restarted GMRES run per instance in lockstep: the host keeps each
// instance's iteration state (Hessenberg matrix, Givens rotations, step
// length) and an instance leaves a loop as soon as its own test says so, so
// its arithmetic is the same alone or in any mix.
//
// The server (bsw_server_s) owns one engine per (order, precision, restart
// length), a FIFO of submitted requests and a worker thread.  Between steps
// it admits queued requests while their device footprint fits the budget and
// a slot is free, and retires finished ones (result copied to host memory,
// device memory released): continuous batching at time-step granularity.
#pragma once

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "bsw_batch_kernels.hpp"

// ====================================================================== engine
namespace {

enum BSlot { B_W = 0, B_BOLD, B_R, B_RT, B_RHS, B_DW, B_WT, B_WK, B_Z, B_U, B_V0 };
constexpr int kBaseSlots = B_V0;

template <class T, class F>
int dispatch2(int P, F& f) {
  switch (P) {
    case 1: return f.template operator()<2, 1, T>();
    case 2: return f.template operator()<2, 2, T>();
    case 3: return f.template operator()<2, 3, T>();
  }
  return BSW_E_ARG;
}

int tri_np(int P) { return (P + 1) * (P + 2) / 2; }
int tri_eb(int P) {  // elements per workgroup of the blocked element kernels
  switch (P) {
    case 1: return Blk<2, 1>::EB;
    case 2: return Blk<2, 2>::EB;
    case 3: return Blk<2, 3>::EB;
  }
  return 1;
}
int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Device bytes one resident 2-D instance takes: state and Krylov vectors,
// diagonal blocks and their inverses, reduction partials, mesh arrays.
int64_t instance_bytes(int64_t n_el, int P, int precision, int M) {
  const int64_t w = precision == BSW_FP64 ? 8 : 4;
  const int64_t bs = 7 * tri_np(P);
  const int64_t len = bs * n_el;
  const int64_t ld = round_up(len, 64);
  const int64_t ntile = (len + kVT - 1) / kVT, ntile_e = (n_el + 255) / 256;
  int64_t b = (kBaseSlots + M + 1) * ld * w;
  b += 2 * bs * bs * n_el * w;
  b += 3 * 7 * 3 * (P + 1) * n_el * w;  // face traces
  b += std::max<int64_t>(66 * ntile, 4 * ntile_e) * 8;
  b += n_el * (3 * 4 + 6 * 8 + 14 * 8 + (precision == BSW_FP32 ? 14 * 4 : 0));
  return b + 4096;
}

struct Request;

template <class T>
struct BInst {
  Request* req = nullptr;
  int slot = -1;
  bsw_mesh mesh = nullptr;
  bsw_disc disc = nullptr;
  T* ws = nullptr;
  int64_t n_el = 0, len = 0, ld = 0;
  int ntile = 0, ntile_e = 0;
  double* part = nullptr;
  bsw_params prm{};
  bsw_solve_opts opt{};
  double newton_tol = 0, gmres_rtol = 0;
  double dt = 0, dtk = 0, t = 0, mass_cur = 0, active_cur = 0;
  int step = 0, nsteps = 0, n_total = 0;
  bool failed = false, cancelled = false;
  bsw_solve_stats st{};
  // Newton / backtracking
  int it = 0, conv = 0;
  double rn = 0, rn_prev = 0, eta = 1e-3, a = 1, rnt = 0;
  // GMRES
  std::vector<double> H, cs, sn, g, y;
  int j = 0, iters = 0, cycles = 0;
  double bn = 0, beta = 0, relres = 0, rtol = 0, hn = 0;
  bool fold = true, cyc_conv = false;
  bool finished() const { return failed || cancelled || step >= nsteps; }
};

template <class T>
void free_instance(BInst<T>* I) {
  if (!I) return;
  hfree(I->ws);
  hfree(I->part);
  if (I->disc) bsw_disc_destroy(I->disc);
  if (I->mesh) bsw_mesh_destroy(I->mesh);
  delete I;
}

template <class T>
struct BatchEngine {
  bsw_ctx c = nullptr;
  int P = 0, M = 30, EB = 1, BS = 1;
  BInst<T>* slots[kMaxBatch] = {};
  InstDesc<T>* d_desc = nullptr;  // device
  InstDesc<T>* h_desc = nullptr;  // pinned staging of the descriptors
  double* sc = nullptr;           // device per-instance scalars [kMaxBatch][kScStride]
  double* sch = nullptr;          // pinned, device-mapped mirror of sc
  double* sch_dev = nullptr;
  double* ystage = nullptr;       // pinned staging of Krylov combination weights
  int64_t ticks = 0, launches = 0;

  ~BatchEngine() {
    for (auto& s : slots) { free_instance(s); s = nullptr; }
    hfree(d_desc);
    hfree(sc);
    if (h_desc) (void)hipHostFree(h_desc);
    if (sch) (void)hipHostFree(sch);
    if (ystage) (void)hipHostFree(ystage);
  }

  int init(bsw_ctx ctx, int P_, int M_) {
    c = ctx; P = P_; M = M_;
    EB = tri_eb(P);
    BS = 7 * tri_np(P);
    if (int rc = dev_alloc(c, &d_desc, kMaxBatch)) return rc;
    if (int rc = dev_alloc(c, &sc, (size_t)kMaxBatch * kScStride)) return rc;
    HIPCHK(c, hipHostMalloc((void**)&h_desc, sizeof(InstDesc<T>) * kMaxBatch, hipHostMallocDefault));
    HIPCHK(c, hipHostMalloc((void**)&sch, sizeof(double) * kMaxBatch * kScStride, hipHostMallocMapped));
    HIPCHK(c, hipHostGetDevicePointer((void**)&sch_dev, sch, 0));
    HIPCHK(c, hipHostMalloc((void**)&ystage, sizeof(double) * kMaxBatch * 72, hipHostMallocDefault));
    std::memset(h_desc, 0, sizeof(InstDesc<T>) * kMaxBatch);
    return BSW_OK;
  }

  int resident() const {
    int n = 0;
    for (auto* s : slots) n += s != nullptr;
    return n;
  }
  int free_slot() const {
    for (int k = 0; k < kMaxBatch; ++k)
      if (!slots[k]) return k;
    return -1;
  }

  // ------------------------------------------------------------ launch sets
  enum Kind { K_ETILE, K_E256, K_E1, K_ITEM, K_VEC, K_ONE };
  int tiles_of(const BInst<T>* I, int kind) const {
    switch (kind) {
      case K_ETILE: return (int)((I->n_el + EB - 1) / EB);
      case K_E256: return I->ntile_e;
      case K_E1: return (int)I->n_el;
      case K_ITEM: return (int)((BS * I->n_el + 255) / 256);
      case K_VEC: return I->ntile;
    }
    return 1;
  }
  // fills inst, tile0 and jv (the Krylov index); rows and s are zeroed
  int build(BatchSet& S, const std::vector<int>& L, int kind) const {
    S.n = (int)L.size();
    int tot = 0;
    for (size_t a = 0; a < L.size(); ++a) {
      const BInst<T>* I = slots[L[a]];
      S.inst[a] = (uint16_t)L[a];
      S.tile0[a] = tot;
      S.jv[a] = (uint8_t)I->j;
      S.rows[a] = 0;
      S.s[a] = 0.0;
      tot += tiles_of(I, kind);
    }
    S.tile0[L.size()] = tot;
    return tot;
  }

  int sync() {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return BSW_OK;
  }
  double rd(int slot, int off) const { return ((volatile double*)sch)[(size_t)slot * kScStride + off]; }

  // ------------------------------------------------------------ element stages
  int step_begin(const std::vector<int>& L) {
    BatchSet S;
    const int nt = build(S, L, K_E256);
    if (!nt) return BSW_OK;
    auto f = [&]<int D, int PP, class TT>() -> int {
      hipLaunchKernelGGL((kb_step_begin<D, PP, TT>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, (int)B_W,
                         (int)B_BOLD);
      HIPCHK(c, hipGetLastError());
      return BSW_OK;
    };
    ++launches;
    return dispatch2<T>(P, f);
  }
  // face traces of slot sX into trace set `which` (0 linearisation, 1 residual, 2 Jacobian)
  int trace(const std::vector<int>& L, int sX, int which) {
    BatchSet S;
    const int nt = build(S, L, K_E256);
    if (!nt) return BSW_OK;
    auto f = [&]<int D, int PP, class TT>() -> int {
      hipLaunchKernelGGL((kb_trace<D, PP, TT>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, sX, which);
      HIPCHK(c, hipGetLastError());
      return BSW_OK;
    };
    ++launches;
    return dispatch2<T>(P, f);
  }
  // mode 0: out = R(W; b_old); mode 1: out = J x (each after the trace pass of its argument)
  int elem(int mode, const std::vector<int>& L, int sW, int sX, int sOut) {
    if (int rc = mode == 0 ? trace(L, sW, 1) : trace(L, sX, 2)) return rc;
    BatchSet S;
    const int nt = build(S, L, K_ETILE);
    if (!nt) return BSW_OK;
    auto f = [&]<int D, int PP, class TT>() -> int {
      if (mode == 0)
        hipLaunchKernelGGL((kb_elem<D, PP, TT, 0>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, sW, sX,
                           (int)B_BOLD, sOut);
      else
        hipLaunchKernelGGL((kb_elem<D, PP, TT, 1>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, sW, sX,
                           (int)B_BOLD, sOut);
      HIPCHK(c, hipGetLastError());
      return BSW_OK;
    };
    ++launches;
    return dispatch2<T>(P, f);
  }
  int linearize(const std::vector<int>& L) {
    if (int rc = trace(L, B_W, 0)) return rc;
    BatchSet S;
    const int nt = build(S, L, K_E1);
    if (!nt) return BSW_OK;
    auto f = [&]<int D, int PP, class TT>() -> int {
      using Sh = Shape<D, PP>;
      hipLaunchKernelGGL((kb_jac_columns<D, PP, TT>), dim3(nt), dim3(Sh::BS <= 64 ? 64 : 128), 0, c->stream,
                         d_desc, S, (int)B_W);
      HIPCHK(c, hipGetLastError());
      hipLaunchKernelGGL((kb_block_inverse<Sh::BS, TT>), dim3(nt), dim3(64), 0, c->stream, d_desc, S);
      HIPCHK(c, hipGetLastError());
      return BSW_OK;
    };
    launches += 2;
    return dispatch2<T>(P, f);
  }
  int prec(const std::vector<int>& L, int sX, int sY) {
    BatchSet S;
    const int nt = build(S, L, K_ITEM);
    if (!nt) return BSW_OK;
    auto f = [&]<int D, int PP, class TT>() -> int {
      using Sh = Shape<D, PP>;
      hipLaunchKernelGGL((kb_block_apply<Sh::BS, TT>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, sX, sY);
      HIPCHK(c, hipGetLastError());
      return BSW_OK;
    };
    ++launches;
    return dispatch2<T>(P, f);
  }

  // ------------------------------------------------------------ vector stages
  // y = a x + b z (flags as kb_lin); s[] gives the per-instance scalar
  int lin(const std::vector<int>& L, int sy, int sx, int sz, double a, double b, int flags,
          const std::vector<double>* s = nullptr) {
    BatchSet S;
    const int nt = build(S, L, K_VEC);
    if (!nt) return BSW_OK;
    if (s)
      for (size_t k = 0; k < L.size(); ++k) S.s[k] = (*s)[k];
    hipLaunchKernelGGL((kb_lin<T>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, sy, sx, sz, a, b, flags);
    HIPCHK(c, hipGetLastError());
    ++launches;
    return BSW_OK;
  }
  int combine(const std::vector<int>& L, const std::vector<int>& rows, int coff, int sw, int sy, double sgn,
              int flags, const std::vector<double>* s = nullptr) {
    BatchSet S;
    const int nt = build(S, L, K_VEC);
    if (!nt) return BSW_OK;
    for (size_t k = 0; k < L.size(); ++k) {
      S.rows[k] = (uint8_t)rows[k];
      if (s) S.s[k] = (*s)[k];
    }
    hipLaunchKernelGGL((kb_combine<T>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, (const double*)sc, coff,
                       (int)B_V0, sw, sy, sgn, flags);
    HIPCHK(c, hipGetLastError());
    ++launches;
    return BSW_OK;
  }
  // fold the partials of rows[] rows per instance into sc / sch at offset off
  int final_rows(const std::vector<int>& L, const std::vector<int>& rows, int etile, unsigned ops, int off) {
    BatchSet S;
    build(S, L, K_ONE);
    int mr = 0;
    for (size_t k = 0; k < L.size(); ++k) {
      S.rows[k] = (uint8_t)rows[k];
      mr = std::max(mr, rows[k]);
    }
    if (!mr) return BSW_OK;
    hipLaunchKernelGGL((kb_rows_final<T>), dim3((unsigned)L.size(), mr), dim3(256), 0, c->stream, d_desc, S, etile,
                       ops, sc, sch_dev, off);
    HIPCHK(c, hipGetLastError());
    ++launches;
    return BSW_OK;
  }
  // V_r . w for r < rows[k] - self, plus w . w as the last row when self
  int multidot(const std::vector<int>& L, const std::vector<int>& rows, int sw, int self, int off) {
    BatchSet S;
    const int nt = build(S, L, K_VEC);
    if (!nt) return BSW_OK;
    int mr = 0;
    for (size_t k = 0; k < L.size(); ++k) {
      S.rows[k] = (uint8_t)rows[k];
      mr = std::max(mr, rows[k]);
    }
    hipLaunchKernelGGL((kb_multidot<T>), dim3(nt, mr), dim3(256), 0, c->stream, d_desc, S, (int)B_V0, sw, self);
    HIPCHK(c, hipGetLastError());
    ++launches;
    return final_rows(L, rows, 0, 0u, off);
  }
  // op 0: sum of squares, 1: max |x|, of slot s0 (and s1 >= 0) -> rows 0 (1) at off
  int vred(const std::vector<int>& L, int s0, int s1, int op, int off) {
    BatchSet S;
    const int nt = build(S, L, K_VEC);
    if (!nt) return BSW_OK;
    const int nr = s1 >= 0 ? 2 : 1;
    hipLaunchKernelGGL((kb_vred<T>), dim3(nt, nr), dim3(256), 0, c->stream, d_desc, S, s0, s1 >= 0 ? s1 : s0, op);
    HIPCHK(c, hipGetLastError());
    ++launches;
    std::vector<int> rows(L.size(), nr);
    const unsigned ops = op == 0 ? 0u : (1u | (1u << 2));
    return final_rows(L, rows, 0, ops, off);
  }
  int diag(const std::vector<int>& L) {
    BatchSet S;
    const int nt = build(S, L, K_E256);
    if (!nt) return BSW_OK;
    auto f = [&]<int D, int PP, class TT>() -> int {
      hipLaunchKernelGGL((kb_diag<D, PP, TT>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, (int)B_W);
      HIPCHK(c, hipGetLastError());
      return BSW_OK;
    };
    ++launches;
    if (int rc = dispatch2<T>(P, f)) return rc;
    std::vector<int> rows(L.size(), 4);
    return final_rows(L, rows, 1, 0u | (0u << 2) | (1u << 4) | (2u << 6), kScB);
  }

  // ------------------------------------------------------------ descriptors
  void fill_desc(int k) {
    BInst<T>* I = slots[k];
    InstDesc<T>& d = h_desc[k];
    d.m = view<T>(I->disc);
    d.p = devparams<T>(I->prm, I->dtk > 0 ? I->dtk : I->dt);
    d.ws = I->ws;
    d.ld = I->ld;
    d.len = I->len;
    d.blk = (T*)I->disc->blocks;
    d.blk_raw = (T*)I->disc->blocks_raw;
    d.trL = (T*)I->disc->trL;
    d.trA = (T*)I->disc->trA;
    d.trX = (T*)I->disc->trX;
    d.part = I->part;
    d.ntile = I->ntile;
    d.ntile_e = I->ntile_e;
  }
  // the pinned staging is only rewritten after a stream synchronisation
  int upload_desc() {
    HIPCHK(c, hipMemcpyAsync(d_desc, h_desc, sizeof(InstDesc<T>) * kMaxBatch, hipMemcpyHostToDevice, c->stream));
    return BSW_OK;
  }

  // ------------------------------------------------------------ admission
  // takes ownership of I; its device arrays are allocated here
  int add(BInst<T>* I, const void* W0_host, const bsw_ic* ic) {
    const int k = free_slot();
    if (k < 0) return fail(c, BSW_E_STATE, "batch is full");
    bsw_disc d = I->disc;
    I->n_el = d->mesh->n_el;
    I->len = bsw_state_len(d);
    I->ld = round_up(I->len, 64);
    I->ntile = (int)((I->len + kVT - 1) / kVT);
    I->ntile_e = (int)((I->n_el + 255) / 256);
    const size_t nb = (size_t)BS * BS * I->n_el;
    if (hipMalloc((void**)&I->ws, sizeof(T) * (size_t)(kBaseSlots + M + 1) * I->ld) != hipSuccess ||
        hipMalloc(&d->blocks, nb * sizeof(T)) != hipSuccess || hipMalloc(&d->blocks_raw, nb * sizeof(T)) != hipSuccess)
      return fail(c, BSW_E_OOM, "instance storage");
    if (int rc = dev_alloc(c, &I->part, (size_t)std::max<int64_t>(66 * I->ntile, 4 * I->ntile_e))) return rc;
    T* W = I->ws + (size_t)B_W * I->ld;
    if (W0_host) {
      HIPCHK(c, hipMemcpyAsync(W, W0_host, sizeof(T) * I->len, hipMemcpyHostToDevice, c->stream));
    } else {
      if (int rc = bsw_project_ic(d, ic, W)) return rc;
    }
    double dg[4];
    if (int rc = bsw_diagnostics(d, &I->prm, W, dg)) return rc;
    std::memset(&I->st, 0, sizeof(I->st));
    I->st.mass0 = dg[0];
    I->mass_cur = dg[0];
    I->active_cur = dg[1];
    const bsw_solve_opts& o = I->opt;
    I->dt = o.dt > 0 ? o.dt : o.cfl * d->mesh->hmin / dg[2];
    if (!(I->dt > 0) || !std::isfinite(I->dt)) return fail(c, BSW_E_ARG, "time step is not positive and finite");
    const double nt = std::ceil(o.t_end / I->dt - 1e-12);
    if (!(nt <= 2.0e9)) return fail(c, BSW_E_ARG, "t_end / dt exceeds 2e9 steps");
    I->n_total = std::max(1, (int)nt);
    I->nsteps = o.max_steps < 0 ? I->n_total : std::min(I->n_total, o.max_steps);
    I->st.dt = I->dt;
    const double floor_tol = sizeof(T) == 4 ? 2e-6 : 0.0;
    I->newton_tol = std::max(o.newton_tol, floor_tol);
    I->gmres_rtol = std::max(o.gmres_rtol, sizeof(T) == 4 ? 1e-6 : 0.0);
    I->H.assign((size_t)(M + 1) * M, 0.0);
    I->cs.assign(M, 0.0);
    I->sn.assign(M, 0.0);
    I->g.assign(M + 1, 0.0);
    I->y.assign(M, 0.0);
    HIPCHK(c, hipStreamSynchronize(c->stream));  // staging below is reused
    I->slot = k;
    slots[k] = I;
    fill_desc(k);
    return BSW_OK;
  }
  // removes the instance from the batch without freeing it
  BInst<T>* take(int k) {
    BInst<T>* I = slots[k];
    slots[k] = nullptr;
    std::memset(&h_desc[k], 0, sizeof(InstDesc<T>));
    return I;
  }

  // ------------------------------------------------------------ GMRES (lockstep)
  // Right-preconditioned restarted GMRES(M) with classical Gram-Schmidt done
  // twice, per instance: J x = rhs to ||rhs - J x|| <= rtol ||rhs||, x = B_DW
  // starting at 0.  The folded norm ||w - V h2||^2 = w.w - |h2|^2 is used
  // unless it cancels, then the norm is taken explicitly.
  int gmres(const std::vector<int>& N) {
    if (int rc = lin(N, B_DW, B_DW, B_DW, 0.0, 0.0, 4)) return rc;
    if (int rc = vred(N, B_RHS, -1, 0, kScB)) return rc;
    if (int rc = sync()) return rc;
    std::vector<int> G;
    std::vector<double> s;
    for (int k : N) {
      BInst<T>* I = slots[k];
      I->iters = 0;
      I->cycles = 0;
      I->relres = 0.0;
      I->bn = std::sqrt(rd(k, kScB));
      I->beta = I->bn;
      if (I->bn > 0.0) {
        G.push_back(k);
        s.push_back(1.0 / I->bn);
      }
    }
    if (int rc = lin(G, B_V0, B_RHS, B_RHS, 0.0, 0.0, 1 | 8, &s)) return rc;
    for (int k : G) {
      BInst<T>* I = slots[k];
      I->j = 0;
      std::fill(I->g.begin(), I->g.end(), 0.0);
      I->g[0] = I->beta;
    }
    std::vector<int> rows, F, E, Rs, keep;
    while (!G.empty()) {
      ++ticks;
      // Arnoldi step of every instance at its own index j
      if (int rc = prec(G, B_V0 | kSlotJ, B_Z)) return rc;
      if (int rc = elem(1, G, B_W, B_Z, B_WK)) return rc;
      rows.clear();
      for (int k : G) {
        slots[k]->iters += 1;
        rows.push_back(slots[k]->j + 1);
      }
      if (int rc = multidot(G, rows, B_WK, 0, kScA)) return rc;
      if (int rc = combine(G, rows, kScA, B_WK, B_WK, -1.0, 4)) return rc;
      for (auto& r : rows) r += 1;
      if (int rc = multidot(G, rows, B_WK, 1, kScB)) return rc;
      if (int rc = sync()) return rc;
      F.clear();
      for (int k : G) {
        BInst<T>* I = slots[k];
        const int j = I->j;
        double hh = 0.0;
        for (int i = 0; i <= j; ++i) {
          const double h2 = rd(k, kScB + i);
          I->H[(size_t)i * M + j] = rd(k, kScA + i) + h2;
          hh += h2 * h2;
        }
        const double ww = rd(k, kScB + j + 1);
        I->fold = hh <= 1e-4 * ww;
        if (I->fold) I->hn = std::sqrt(std::max(ww - hh, 0.0));
        else F.push_back(k);
      }
      if (!F.empty()) {
        std::vector<int> fr;
        for (int k : F) fr.push_back(slots[k]->j + 1);
        if (int rc = combine(F, fr, kScB, B_WK, B_WK, -1.0, 4)) return rc;
        if (int rc = vred(F, B_WK, -1, 0, kScA)) return rc;
        if (int rc = sync()) return rc;
        for (int k : F) slots[k]->hn = std::sqrt(rd(k, kScA));
      }
      // V_{j+1} = (w - V h2) / hn  (the subtraction already done where not folded)
      rows.clear();
      s.clear();
      for (int k : G) {
        BInst<T>* I = slots[k];
        rows.push_back(I->fold ? I->j + 1 : 0);
        s.push_back(I->hn > 0.0 ? 1.0 / I->hn : 0.0);
      }
      if (int rc = combine(G, rows, kScB, B_WK, (B_V0 + 1) | kSlotJ, 1.0, 1, &s)) return rc;
      // Givens rotations and the cycle test, per instance
      E.clear();
      keep.clear();
      for (int k : G) {
        BInst<T>* I = slots[k];
        const int j = I->j;
        double* H = I->H.data();
        H[(size_t)(j + 1) * M + j] = I->hn;
        for (int i = 0; i < j; ++i) {
          const double t = I->cs[i] * H[(size_t)i * M + j] + I->sn[i] * H[(size_t)(i + 1) * M + j];
          H[(size_t)(i + 1) * M + j] = -I->sn[i] * H[(size_t)i * M + j] + I->cs[i] * H[(size_t)(i + 1) * M + j];
          H[(size_t)i * M + j] = t;
        }
        const double den = std::hypot(H[(size_t)j * M + j], H[(size_t)(j + 1) * M + j]);
        I->cs[j] = H[(size_t)j * M + j] / den;
        I->sn[j] = H[(size_t)(j + 1) * M + j] / den;
        H[(size_t)j * M + j] = den;
        H[(size_t)(j + 1) * M + j] = 0.0;
        I->g[j + 1] = -I->sn[j] * I->g[j];
        I->g[j] = I->cs[j] * I->g[j];
        I->cyc_conv = std::fabs(I->g[j + 1]) <= I->rtol * I->bn || I->hn == 0.0;
        I->j = j + 1;
        if (I->cyc_conv || I->j == M || I->iters >= I->opt.gmres_max_iters) E.push_back(k);
        else keep.push_back(k);
      }
      if (E.empty()) continue;
      // cycle end: x += M^{-1} V y, then the true residual rhs - J x -> V_0
      rows.clear();
      for (int k : E) {
        BInst<T>* I = slots[k];
        const int jj = I->j;
        const double* H = I->H.data();
        for (int i = jj - 1; i >= 0; --i) {
          double t = I->g[i];
          for (int q = i + 1; q < jj; ++q) t -= H[(size_t)i * M + q] * I->y[q];
          I->y[i] = t / H[(size_t)i * M + i];
        }
        double* st = ystage + (size_t)k * 72;
        for (int i = 0; i < jj; ++i) st[i] = I->y[i];
        HIPCHK(c, hipMemcpyAsync(sc + (size_t)k * kScStride + kScA, st, sizeof(double) * jj, hipMemcpyHostToDevice,
                                 c->stream));
        rows.push_back(jj);
        I->cycles += 1;
      }
      if (int rc = combine(E, rows, kScA, B_WK, B_Z, 1.0, 2)) return rc;
      if (int rc = prec(E, B_Z, B_U)) return rc;
      if (int rc = lin(E, B_DW, B_DW, B_U, 1.0, 1.0, 0)) return rc;
      if (int rc = elem(1, E, B_W, B_DW, B_WK)) return rc;
      if (int rc = lin(E, B_V0, B_RHS, B_WK, 1.0, -1.0, 0)) return rc;
      if (int rc = vred(E, B_V0, -1, 0, kScB)) return rc;
      if (int rc = sync()) return rc;
      Rs.clear();
      s.clear();
      for (int k : E) {
        BInst<T>* I = slots[k];
        I->beta = std::sqrt(rd(k, kScB));
        I->relres = I->beta / I->bn;
        if (I->cyc_conv || I->beta <= I->rtol * I->bn || I->iters >= I->opt.gmres_max_iters) continue;
        Rs.push_back(k);
        s.push_back(1.0 / I->beta);
        I->j = 0;
        std::fill(I->g.begin(), I->g.end(), 0.0);
        I->g[0] = I->beta;
      }
      if (int rc = lin(Rs, B_V0, B_V0, B_V0, 0.0, 0.0, 1 | 8, &s)) return rc;
      G = keep;
      G.insert(G.end(), Rs.begin(), Rs.end());
      std::sort(G.begin(), G.end());
    }
    return BSW_OK;
  }

  // ------------------------------------------------------------ one time step
  int step_all() {
    std::vector<int> S;
    for (int k = 0; k < kMaxBatch; ++k)
      if (slots[k] && !slots[k]->finished()) S.push_back(k);
    if (S.empty()) return BSW_OK;
    for (int k : S) {
      BInst<T>* I = slots[k];
      const int kk = I->step + 1;
      I->dtk = kk < I->n_total ? I->dt : I->opt.t_end - (kk - 1) * I->dt;
      fill_desc(k);
    }
    if (int rc = upload_desc()) return rc;
    if (int rc = step_begin(S)) return rc;
    if (int rc = elem(0, S, B_W, B_W, B_R)) return rc;
    if (int rc = vred(S, B_R, -1, 0, kScB)) return rc;
    if (int rc = sync()) return rc;
    for (int k : S) {
      BInst<T>* I = slots[k];
      I->st.operator_applies += 1;
      I->rn = std::sqrt(rd(k, kScB));
      I->rn_prev = I->rn;
      I->it = 0;
      I->conv = 0;
      I->eta = 1e-3;
    }
    std::vector<int> N = S, C, L, A, nxt;
    std::vector<double> s;
    while (!N.empty()) {
      for (int k : N) {
        BInst<T>* I = slots[k];
        I->it += 1;
        // Eisenstat-Walker forcing (choice 2, gamma 0.9, exponent 2) in [gmres_rtol, 1e-3]
        if (I->it > 1) {
          const double r = I->rn / std::max(I->rn_prev, 1e-300);
          const double cand = 0.9 * r * r, safe = 0.9 * I->eta * I->eta;
          I->eta = std::max(cand, safe > 0.1 ? safe : 0.0);
        }
        I->eta = std::min(1e-3, std::max(I->eta, I->gmres_rtol));
        I->rtol = I->eta;
      }
      if (int rc = linearize(N)) return rc;
      if (int rc = lin(N, B_RHS, B_R, B_R, -1.0, 0.0, 8)) return rc;
      if (int rc = gmres(N)) return rc;
      for (int k : N) {
        BInst<T>* I = slots[k];
        I->st.gmres_total += I->iters;
        I->st.jacobian_applies += I->iters + I->cycles;
      }
      // Newton test on the full update
      if (int rc = vred(N, B_DW, B_W, 1, kScB)) return rc;
      if (int rc = sync()) return rc;
      C.clear();
      L.clear();
      for (int k : N) {
        const double nd = rd(k, kScB), nw = rd(k, kScB + 1);
        if (std::isfinite(nd) && nd <= slots[k]->newton_tol * (1.0 + nw)) {
          slots[k]->conv = 1;
          C.push_back(k);
        } else {
          slots[k]->a = 1.0;
          L.push_back(k);
        }
      }
      if (int rc = lin(C, B_W, B_W, B_DW, 1.0, 1.0, 0)) return rc;
      // backtracking on ||R||
      while (!L.empty()) {
        s.clear();
        for (int k : L) s.push_back(slots[k]->a);
        if (int rc = lin(L, B_WT, B_W, B_DW, 1.0, 0.0, 2, &s)) return rc;
        if (int rc = elem(0, L, B_WT, B_WT, B_RT)) return rc;
        if (int rc = vred(L, B_RT, -1, 0, kScB)) return rc;
        if (int rc = sync()) return rc;
        A.clear();
        nxt.clear();
        for (int k : L) {
          BInst<T>* I = slots[k];
          I->st.operator_applies += 1;
          I->rnt = std::sqrt(rd(k, kScB));
          if ((std::isfinite(I->rnt) && I->rnt <= (1.0 - 1e-4 * I->a) * I->rn) || I->a <= 1.0 / 64.0) {
            A.push_back(k);
          } else {
            I->a *= 0.5;
            nxt.push_back(k);
          }
        }
        if (int rc = lin(A, B_W, B_WT, B_WT, 1.0, 0.0, 8)) return rc;
        if (int rc = lin(A, B_R, B_RT, B_RT, 1.0, 0.0, 8)) return rc;
        for (int k : A) {
          BInst<T>* I = slots[k];
          I->rn_prev = I->rn;
          I->rn = I->rnt;
          if (!std::isfinite(I->rnt)) I->conv = -1;
        }
        L = nxt;
      }
      nxt.clear();
      for (int k : N)
        if (slots[k]->conv == 0 && slots[k]->it < slots[k]->opt.max_newton) nxt.push_back(k);
      N = nxt;
    }
    if (int rc = diag(S)) return rc;
    if (int rc = sync()) return rc;
    for (int k : S) {
      BInst<T>* I = slots[k];
      I->st.newton_total += I->it;
      I->st.newton_max = std::max(I->st.newton_max, I->it);
      if (I->conv != 1) {
        I->st.capped += 1;
        I->st.status = BSW_W_NOT_CONVERGED;
      }
      I->mass_cur = rd(k, kScB);
      I->active_cur = 100.0 * rd(k, kScB + 1) / I->disc->mesh->measure;
      I->st.max_mass_drift = std::max(I->st.max_mass_drift, std::fabs(I->mass_cur - I->st.mass0) / I->st.mass0);
      I->t += I->dtk;
      I->step += 1;
      I->st.steps = I->step;
      if (I->conv < 0) I->failed = true;
    }
    return BSW_OK;
  }

  // final statistics of a finished instance
  void final_stats(BInst<T>* I) {
    I->st.mass_end = I->mass_cur;
    I->st.active_pct = I->active_cur;
    I->st.t_end = I->t;
  }
};

}  // namespace

// ====================================================================== server
namespace {

struct Request {
  uint64_t ticket = 0;
  std::atomic<int> state{BSW_REQ_QUEUED};
  int next_state = BSW_REQ_DONE;  // set by the engine, published under the server lock
  std::atomic<bool> cancel{false};
  int P = 0, precision = 0, M = 30;
  int64_t n_vert = 0, n_el = 0, footprint = 0;
  std::vector<double> xy;
  std::vector<int32_t> e2v;
  std::vector<unsigned char> W0;  // optional initial state (host copy)
  bsw_params prm{};
  bsw_ic ic{};
  bsw_solve_opts opt{};
  std::vector<unsigned char> W;   // result (host copy)
  bsw_solve_stats st{};
  int rc = BSW_OK;
  std::string err;
  std::chrono::steady_clock::time_point t_submit, t_start, t_end;
};

struct EngineIf {
  virtual ~EngineIf() = default;
  virtual int admit(Request* r, std::string& err) = 0;
  virtual int step() = 0;
  // detaches finished or cancelled instances: result to host, device memory freed
  virtual void retire(std::vector<Request*>& out) = 0;
  // detaches every instance after a device error
  virtual void drop_all(std::vector<Request*>& out) = 0;
  virtual int resident() const = 0;
  virtual bool has_free() const = 0;
  virtual int64_t launches() const = 0;
};

template <class T>
struct EngineImpl final : EngineIf {
  BatchEngine<T> e;
  int admit(Request* r, std::string& err) override {
    bsw_ctx c = e.c;
    BInst<T>* I = new BInst<T>();
    I->req = r;
    I->prm = r->prm;
    I->opt = r->opt;
    int rc = bsw_mesh_upload(c, 2, r->n_vert, r->xy.data(), r->n_el, r->e2v.data(), &I->mesh);
    if (!rc) rc = bsw_disc_create(I->mesh, r->P, r->precision, &I->disc);
    if (!rc) rc = check_params(I->disc, &I->prm);
    if (!rc) rc = e.add(I, r->W0.empty() ? nullptr : r->W0.data(), &r->ic);
    if (rc) {
      err = c->err;
      free_instance(I);
    }
    return rc;
  }
  int step() override { return e.step_all(); }
  void retire(std::vector<Request*>& out) override {
    for (int k = 0; k < kMaxBatch; ++k) {
      BInst<T>* I = e.slots[k];
      if (!I) continue;
      Request* r = I->req;
      const bool cancel = r->cancel.load();
      if (!I->finished() && !cancel) continue;
      e.take(k);
      if (cancel && !I->finished()) {
        r->next_state = BSW_REQ_CANCELLED;
      } else {
        r->W.resize(sizeof(T) * I->len);
        const hipError_t he = hipMemcpy(r->W.data(), I->ws + (size_t)B_W * I->ld, sizeof(T) * I->len,
                                        hipMemcpyDeviceToHost);
        e.final_stats(I);
        r->st = I->st;
        if (he != hipSuccess) {
          r->rc = BSW_E_HIP;
          r->err = std::string("result copy: ") + hipGetErrorString(he);
          r->next_state = BSW_REQ_FAILED;
        } else {
          r->rc = I->st.status;
          r->next_state = BSW_REQ_DONE;
        }
      }
      free_instance(I);
      out.push_back(r);
    }
  }
  void drop_all(std::vector<Request*>& out) override {
    for (int k = 0; k < kMaxBatch; ++k) {
      BInst<T>* I = e.slots[k];
      if (!I) continue;
      e.take(k);
      out.push_back(I->req);
      free_instance(I);
    }
  }
  int resident() const override { return e.resident(); }
  bool has_free() const override { return e.free_slot() >= 0; }
  int64_t launches() const override { return e.launches; }
};

}  // namespace

struct bsw_server_s {
  bsw_ctx user = nullptr;
  bsw_ctx_s ictx;                 // the server's own context and stream
  size_t budget = 0;
  int max_slots = 0;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<Request*> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::map<long, std::unique_ptr<EngineIf>> engines;  // key: (P, precision, M)
  uint64_t next_ticket = 1;
  int64_t in_use = 0;
  int resident = 0, peak_resident = 0;
  int64_t steps = 0, completed = 0;
  bool stop = false;
  std::thread th;

  static long key(const Request* r) { return ((long)r->P * 4 + r->precision) * 256 + r->M; }

  EngineIf* engine_for(const Request* r, std::string& err) {
    auto it = engines.find(key(r));
    if (it != engines.end()) return it->second.get();
    std::unique_ptr<EngineIf> E;
    int rc;
    if (r->precision == BSW_FP64) {
      auto* x = new EngineImpl<double>();
      E.reset(x);
      rc = x->e.init(&ictx, r->P, r->M);
    } else {
      auto* x = new EngineImpl<float>();
      E.reset(x);
      rc = x->e.init(&ictx, r->P, r->M);
    }
    if (rc) {
      err = ictx.err;
      return nullptr;
    }
    EngineIf* p = E.get();
    engines[key(r)] = std::move(E);
    return p;
  }

  void finish(Request* r) {  // under mu
    r->t_end = std::chrono::steady_clock::now();
    r->st.queue_seconds = std::chrono::duration<double>(r->t_start - r->t_submit).count();
    r->st.seconds = std::chrono::duration<double>(r->t_end - r->t_start).count();
    in_use -= r->footprint;
    resident -= 1;
    completed += 1;
  }

  void run() {
    (void)hipSetDevice(ictx.device);
    std::vector<Request*> adm, out;
    for (;;) {
      adm.clear();
      {
        std::unique_lock<std::mutex> lk(mu);
        if (stop) break;
        for (auto it = queue.begin(); it != queue.end();) {
          if ((*it)->cancel.load()) {
            (*it)->state = BSW_REQ_CANCELLED;
            it = queue.erase(it);
            cv_done.notify_all();
          } else {
            ++it;
          }
        }
        // FIFO admission by footprint and slots
        while (!queue.empty()) {
          Request* r = queue.front();
          if (resident >= max_slots || in_use + r->footprint > (int64_t)budget) break;
          std::string err;
          EngineIf* E = engine_for(r, err);
          if (!E) {
            queue.pop_front();
            r->rc = BSW_E_HIP;
            r->err = err;
            r->state = BSW_REQ_FAILED;
            cv_done.notify_all();
            continue;
          }
          if (!E->has_free()) break;
          queue.pop_front();
          resident += 1;
          in_use += r->footprint;
          peak_resident = std::max(peak_resident, resident);
          r->t_start = std::chrono::steady_clock::now();
          r->state = BSW_REQ_RUNNING;
          adm.push_back(r);
        }
        if (adm.empty() && resident == 0) {
          cv.wait_for(lk, std::chrono::milliseconds(20));
          continue;
        }
      }
      for (Request* r : adm) {
        std::string err;
        EngineIf* E;
        {
          std::lock_guard<std::mutex> lk(mu);
          E = engines[key(r)].get();
        }
        const int rc = E->admit(r, err);
        if (rc) {
          std::lock_guard<std::mutex> lk(mu);
          r->rc = rc;
          r->err = err;
          finish(r);
          completed -= 1;
          r->state = BSW_REQ_FAILED;
          cv_done.notify_all();
        }
      }
      for (auto& kv : engines) {
        EngineIf* E = kv.second.get();
        if (!E->resident()) continue;
        out.clear();
        const int rc = E->step();
        if (rc < 0) {
          const std::string err = ictx.err;
          E->drop_all(out);
          std::lock_guard<std::mutex> lk(mu);
          for (Request* r : out) {
            r->rc = rc;
            r->err = err;
            finish(r);
            r->state = BSW_REQ_FAILED;
          }
          cv_done.notify_all();
          continue;
        }
        E->retire(out);
        std::lock_guard<std::mutex> lk(mu);
        steps += 1;
        for (Request* r : out) {
          finish(r);
          r->state = r->next_state;
        }
        if (!out.empty()) cv_done.notify_all();
      }
    }
  }
};

namespace {
bool terminal(int s) { return s == BSW_REQ_DONE || s == BSW_REQ_FAILED || s == BSW_REQ_CANCELLED; }

int check_request(bsw_ctx c, const bsw_solve_request* q) {
  if (!q || !q->xy || !q->el2vert) return fail(c, BSW_E_ARG, "null request or mesh arrays");
  if (q->P < 1 || q->P > 3) return fail(c, BSW_E_ARG, "served solves are 2-D with P in 1..3");
  if (q->precision != BSW_FP64 && q->precision != BSW_FP32) return fail(c, BSW_E_ARG, "bad precision");
  if (q->n_vert < 3 || q->n_el < 1 || q->n_el > (int64_t(1) << 29)) return fail(c, BSW_E_ARG, "bad mesh sizes");
  const bsw_solve_opts& o = q->opts;
  if (o.max_newton < 1 || o.gmres_max_iters < 1 || !(o.t_end > 0) || o.gmres_m < 1 || o.gmres_m > 64)
    return fail(c, BSW_E_ARG, "bad solve options");
  if (!(o.dt > 0) && !(o.cfl > 0)) return fail(c, BSW_E_ARG, "need dt > 0 or cfl > 0");
  const bsw_params* p = &q->params;
  if (p->reg < 1 || p->reg > 3 || p->bc < 1 || p->bc > 3) return fail(c, BSW_E_ARG, "bad reg or bc");
  if (!(p->g > 0) || !(p->rho > 0) || p->eta < 0 || p->sigma0 < 0 || !(p->gamma > 0) || !(p->beta > 0))
    return fail(c, BSW_E_ARG, "need g, rho, gamma, beta > 0 and eta, sigma0 >= 0");
  if (p->reg != 3 && p->sigma0 > 0 && p->sigma0 < 0.5 / p->beta)
    return fail(c, BSW_E_ARG, "regularisations 1 and 2 need sigma0 >= 1/(2 beta)");
  return BSW_OK;
}
}  // namespace

extern "C" {

int64_t bsw_request_footprint(const bsw_solve_request* q) {
  if (!q || q->P < 1 || q->P > 3 || q->n_el < 1) return -1;
  return instance_bytes(q->n_el, q->P, q->precision, std::max(1, std::min(64, q->opts.gmres_m)));
}

int bsw_server_create(bsw_ctx ctx, size_t hbm_budget_bytes, int max_slots, bsw_server* out) {
  if (!ctx || !out) return fail(ctx, BSW_E_ARG, "null argument");
  if (max_slots < 1 || hbm_budget_bytes == 0) return fail(ctx, BSW_E_ARG, "need max_slots >= 1 and a budget");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  auto* S = new bsw_server_s();
  S->user = ctx;
  S->ictx.device = ctx->device;
  if (hipStreamCreateWithFlags(&S->ictx.stream, hipStreamNonBlocking) != hipSuccess) {
    delete S;
    return fail(ctx, BSW_E_HIP, "hipStreamCreateWithFlags");
  }
  S->budget = hbm_budget_bytes;
  S->max_slots = max_slots;
  S->th = std::thread([S] { S->run(); });
  *out = S;
  return BSW_OK;
}

int bsw_server_destroy(bsw_server S) {
  if (!S) return BSW_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  (void)hipSetDevice(S->ictx.device);
  (void)hipStreamSynchronize(S->ictx.stream);
  S->engines.clear();
  (void)hipStreamDestroy(S->ictx.stream);
  delete S;
  return BSW_OK;
}

int bsw_solve_submit(bsw_server S, const bsw_solve_request* q, uint64_t* ticket) {
  if (!S || !ticket) return fail(S ? S->user : nullptr, BSW_E_ARG, "null argument");
  if (int rc = check_request(S->user, q)) return rc;
  for (int64_t k = 0; k < q->n_el * 3; ++k)
    if (q->el2vert[k] < 0 || q->el2vert[k] >= q->n_vert) return fail(S->user, BSW_E_ARG, "vertex index out of range");
  auto r = std::make_unique<Request>();
  r->P = q->P;
  r->precision = q->precision;
  r->M = q->opts.gmres_m;
  r->n_vert = q->n_vert;
  r->n_el = q->n_el;
  r->xy.assign(q->xy, q->xy + 2 * q->n_vert);
  r->e2v.assign(q->el2vert, q->el2vert + 3 * q->n_el);
  if (q->W0) {
    const size_t bytes = (size_t)7 * tri_np(q->P) * q->n_el * (q->precision == BSW_FP64 ? 8 : 4);
    r->W0.assign((const unsigned char*)q->W0, (const unsigned char*)q->W0 + bytes);
  }
  r->prm = q->params;
  r->ic = q->ic;
  r->opt = q->opts;
  r->footprint = bsw_request_footprint(q);
  if (r->footprint > (int64_t)S->budget) return fail(S->user, BSW_E_ARG, "request footprint exceeds the server budget");
  r->t_submit = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->queue.push_back(r.get());
    S->reqs[r->ticket] = std::move(r);
  }
  S->cv.notify_all();
  return BSW_OK;
}

int bsw_solve_poll(bsw_server S, uint64_t ticket, int* state) {
  if (!S || !state) return fail(S ? S->user : nullptr, BSW_E_ARG, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(S->user, BSW_E_ARG, "unknown ticket");
  *state = it->second->state.load();
  return BSW_OK;
}

int bsw_solve_wait(bsw_server S, uint64_t ticket, double timeout_s, int* state) {
  if (!S || !state) return fail(S ? S->user : nullptr, BSW_E_ARG, "null argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(S->user, BSW_E_ARG, "unknown ticket");
  Request* r = it->second.get();
  const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(std::max(0.0, timeout_s));
  while (!terminal(r->state.load()))
    if (S->cv_done.wait_until(lk, until) == std::cv_status::timeout) break;
  *state = r->state.load();
  return BSW_OK;
}

int bsw_solve_fetch(bsw_server S, uint64_t ticket, void* host_W, bsw_solve_stats* stats) {
  if (!S) return BSW_E_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(S->user, BSW_E_ARG, "unknown ticket");
  Request* r = it->second.get();
  const int st = r->state.load();
  if (!terminal(st)) return fail(S->user, BSW_E_STATE, "request has not finished");
  int rc = r->rc;
  if (st == BSW_REQ_DONE) {
    if (host_W) std::memcpy(host_W, r->W.data(), r->W.size());
    if (stats) *stats = r->st;
  } else if (st == BSW_REQ_CANCELLED) {
    rc = fail(S->user, BSW_E_STATE, "request was cancelled");
  } else {
    rc = fail(S->user, r->rc < 0 ? r->rc : BSW_E_HIP, r->err.empty() ? "request failed" : r->err);
  }
  S->reqs.erase(it);
  return rc;
}

int bsw_solve_cancel(bsw_server S, uint64_t ticket) {
  if (!S) return BSW_E_ARG;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(S->user, BSW_E_ARG, "unknown ticket");
    it->second->cancel = true;
  }
  S->cv.notify_all();
  return BSW_OK;
}

int bsw_server_info(bsw_server S, double* out8) {
  if (!S || !out8) return BSW_E_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  int64_t launches = 0;
  for (auto& kv : S->engines) launches += kv.second->launches();
  out8[0] = (double)S->queue.size();
  out8[1] = (double)S->resident;
  out8[2] = (double)S->in_use;
  out8[3] = (double)S->budget;
  out8[4] = (double)S->steps;
  out8[5] = (double)launches;
  out8[6] = (double)S->completed;
  out8[7] = (double)S->peak_resident;
  return BSW_OK;
}

}  // extern "C"
