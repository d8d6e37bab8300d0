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
// length), each with its own worker thread and HIP stream, and a FIFO of
// submitted requests.  Between steps a worker admits its queued requests while
// their device footprint fits the shared budget and a slot is free, and
// retires finished ones (result copied to host memory, device memory
// released): continuous batching at time-step granularity, batches of
// different engines overlapping on the device.
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

int n_modes(int dim, int P) { return dim == 1 ? P + 1 : (P + 1) * (P + 2) / 2; }
int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ------------------------------------------------------------ tile autotuner
// Picks the element-tile variant of the element pass (elem_tile: on triangles
// the occupancy target, in 1-D the workgroup size) per (dimension, order,
// precision, residual or Jacobian, size class).  The
// first launches of a key rotate through the shapes; the caller brackets each
// with a HIP event pair and hands the pair over once both are recorded.
// Completed pairs are read without blocking (hipEventQuery) on later picks,
// and once every shape has kTunerSamples timings the one with the smallest
// is kept for the process.  All shapes compute the same bits, so the choice
// never changes a result.  policy >= 0 forces one shape.  Engines on several
// threads share the table under its mutex.
constexpr int kTunerSamples = 5;

struct TileTuner {
  struct Entry {
    int choice = -1, next = 0;
    int n[kTileShapes] = {};
    float best_ms[kTileShapes] = {};
  };
  struct Pending {
    uint64_t key;
    int v;
    hipEvent_t a, b;
  };
  std::mutex mu;
  std::map<uint64_t, Entry> tab;
  std::vector<Pending> pend;
  int policy = -1;

  static uint64_t key(int dim, int P, int wbytes, int mode, int64_t n_el) {
    int cls = 0;
    while (cls < 40 && (int64_t(1) << (cls + 1)) <= n_el) ++cls;  // floor(log2 n_el)
    return (uint64_t)dim | (uint64_t)P << 4 | (uint64_t)wbytes << 8 | (uint64_t)mode << 16 | (uint64_t)cls << 24;
  }
  void poll_locked() {
    for (size_t k = 0; k < pend.size();) {
      Pending& q = pend[k];
      if (hipEventQuery(q.b) != hipSuccess) { ++k; continue; }
      float ms = 0.0f;
      // (samples still in flight when the choice was made are dropped, so the
      // table keeps the times the choice was made from)
      Entry& E = tab[q.key];
      if (E.choice < 0 && hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
        if (E.n[q.v] == 0 || ms < E.best_ms[q.v]) E.best_ms[q.v] = ms;
        ++E.n[q.v];
        bool all = true;
        for (int v = 0; v < kTileShapes; ++v) all = all && E.n[v] >= kTunerSamples;
        if (all && E.choice < 0) {
          int b = 0;
          for (int v = 1; v < kTileShapes; ++v)
            if (E.best_ms[v] < E.best_ms[b]) b = v;
          E.choice = b;
        }
      }
      (void)hipEventDestroy(q.a);
      (void)hipEventDestroy(q.b);
      pend[k] = pend.back();
      pend.pop_back();
    }
  }
  // the shape for the next launch of key; *measure tells whether the key is
  // still being measured (then time the launch and call submit)
  int pick(uint64_t k, bool* measure) {
    std::lock_guard<std::mutex> lk(mu);
    *measure = false;
    if (policy >= 0) return policy;
    poll_locked();
    Entry& E = tab[k];
    if (E.choice >= 0) return E.choice;
    const int v = E.next;
    E.next = (E.next + 1) % kTileShapes;
    *measure = true;
    return v;
  }
  // an event pair, both already recorded around a launch of shape v; the
  // table owns and destroys them
  void submit(uint64_t k, int v, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> lk(mu);
    pend.push_back({k, v, a, b});
  }
};

TileTuner& tile_tuner() {
  static TileTuner t;
  return t;
}

int single_call_variant() {
  TileTuner& t = tile_tuner();
  std::lock_guard<std::mutex> lk(t.mu);
  return t.policy;
}

// Device bytes one resident instance takes: state and Krylov vectors,
// diagonal blocks and their FP32 block-Jacobi factors, face traces, reduction
// partials, mesh.
int64_t instance_bytes(int64_t n_el, int dim, int P, int precision, int M) {
  const int64_t w = precision == BSW_FP64 ? 8 : 4;
  const int64_t nf = 1 + dim + dim * dim;
  const int64_t bs = nf * n_modes(dim, P);
  const int64_t nfp = (dim + 1) * (dim == 1 ? 1 : P + 1);
  const int64_t len = bs * n_el;
  const int64_t ld = round_up(len, 64);
  const int64_t ntile = (len + kVT - 1) / kVT, ntile_e = (n_el + 255) / 256;
  int64_t b = (kBaseSlots + M + 1) * ld * w;
  b += bs * bs * n_el * w + (int64_t)schur_numbers(dim, n_modes(dim, P)) * n_el * 4;  // blocks, FP32 factors
  b += nf * nfp * n_el * w;  // face traces of the linearisation state
  b += std::max<int64_t>(std::max<int64_t>(130 * ntile, 4 * ntile_e), 4096) * 8;
  const int64_t geo = dim * dim + 1 + (dim + 1) * (dim + 1);
  b += n_el * ((dim + 1) * 4 + (dim + 1) * dim * 8 + geo * 8 + (precision == BSW_FP32 ? geo * 4 : 0));
  b += n_modes(dim, P) * n_el * w;  // bed coefficients
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
  T* bed = nullptr;  // bed coefficients of a served solve with a variable bed
  int64_t n_el = 0, len = 0, ld = 0;
  int ntile = 0, ntile_e = 0;
  double* part = nullptr;
  bsw_params prm{};
  bsw_solve_opts opt{};
  double newton_tol = 0, gmres_rtol = 0;
  double dt = 0, dtk = 0, t = 0, mass_cur = 0, active_cur = 0;
  int step = 0, nsteps = 0, n_total = 0;
  int stage = 0, nstage = 1;   // continuation stage within the current step
  int it_step = 0;             // Newton iterations of the current step (all stages)
  double bold_norm = 0;        // ||b_old||_2 of the current step (res_tol)
  int gm_ref = 0, gm_last = 0; // GMRES iterations after the last preconditioner build, and last
  bool gm_ok = true, rebuilt = false;
  double gamma_cur = 0;        // gamma of the current stage (0: the parameters' gamma)
  bool failed = false, cancelled = false;
  bsw_solve_stats st{};
  // Newton / backtracking
  int it = 0, conv = 0;
  double rn = 0, rn_prev = 0, eta = 1e-3, a = 1, rnt = 0;
  // GMRES
  // H: Hessenberg columns after the Givens rotations; Hu: the completed
  // columns as formed; Hp: the latest column before its completion
  std::vector<double> H, Hu, Hp, cs, sn, g, y;
  int j = 0, iters = 0, cycles = 0;
  double bn = 0, beta = 0, relres = 0, rtol = 0, hn = 0, gsave = 0;
  bool cyc_conv = false;
  bool own = true;  // mesh, discretisation and workspace belong to the instance
  bool finished() const { return failed || cancelled || step >= nsteps; }
};

template <class T>
void free_instance(BInst<T>* I) {
  if (!I) return;
  if (I->own) {
    hfree(I->ws);
    hfree(I->part);
    hfree(I->bed);
    if (I->disc) bsw_disc_destroy(I->disc);
    if (I->mesh) bsw_mesh_destroy(I->mesh);
  }
  delete I;
}

template <class T>
struct BatchEngine {
  bsw_ctx c = nullptr;
  int dim = 2, P = 0, M = 30, BS = 1, NFNFC = 1;
  int EBv[kTileShapes] = {1, 1, 1};  // elements per element-pass workgroup, per tile shape
  int eb_cur = 1;                    // the shape of the element launch being built
  BInst<T>* slots[kMaxBatch] = {};
  InstDesc<T>* d_desc = nullptr;  // device
  InstDesc<T>* h_desc = nullptr;  // pinned staging of the descriptors
  double* sc = nullptr;           // device per-instance scalars [kMaxBatch][kScStride]
  double* sch = nullptr;          // pinned, device-mapped mirror of sc
  double* sch_dev = nullptr;
  double* ystage = nullptr;       // pinned staging of Krylov combination weights
  T* d_dirtab = nullptr;          // device [kMaxBatch][28]: Dirichlet states of boundary tags 0..3
  T* h_dirtab = nullptr;          // pinned staging of d_dirtab
  std::atomic<int64_t> ticks{0}, launches{0};

  ~BatchEngine() {
    destroy_events();
    for (auto& s : slots) { free_instance(s); s = nullptr; }
    hfree(d_desc);
    hfree(sc);
    if (h_desc) (void)hipHostFree(h_desc);
    if (sch) (void)hipHostFree(sch);
    if (ystage) (void)hipHostFree(ystage);
    hfree(d_dirtab);
    if (h_dirtab) (void)hipHostFree(h_dirtab);
  }

  int init(bsw_ctx ctx, int dim_, int P_, int M_) {
    c = ctx; dim = dim_; P = P_; M = M_;
    auto fs = [&]<int D, int PP, class TT>() -> int {
      EBv[0] = etile_eb<D, PP, 0>();
      EBv[1] = etile_eb<D, PP, 1>();
      EBv[2] = etile_eb<D, PP, 2>();
      BS = Shape<D, PP>::BS;
      NFNFC = Shape<D, PP>::NF * Shape<D, PP>::NFC;
      return BSW_OK;
    };
    if (dispatchT<T>(dim, P, fs)) return fail(c, BSW_E_ARG, "unsupported order for this dimension");
    if (int rc = dev_alloc(c, &d_desc, kMaxBatch)) return rc;
    if (int rc = dev_alloc(c, &sc, (size_t)kMaxBatch * kScStride)) return rc;
    HIPCHK(c, hipHostMalloc((void**)&h_desc, sizeof(InstDesc<T>) * kMaxBatch, hipHostMallocDefault));
    HIPCHK(c, hipHostMalloc((void**)&sch, sizeof(double) * kMaxBatch * kScStride, hipHostMallocMapped));
    HIPCHK(c, hipHostGetDevicePointer((void**)&sch_dev, sch, 0));
    HIPCHK(c, hipHostMalloc((void**)&ystage, sizeof(double) * kMaxBatch * 72, hipHostMallocDefault));
    if (int rc = dev_alloc(c, &d_dirtab, (size_t)kMaxBatch * 28)) return rc;
    HIPCHK(c, hipHostMalloc((void**)&h_dirtab, sizeof(T) * kMaxBatch * 28, hipHostMallocDefault));
    std::memset(h_dirtab, 0, sizeof(T) * kMaxBatch * 28);
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
  enum Kind { K_ETILE, K_E256, K_SCHUR, K_PREC, K_VEC, K_ONE, K_TRACE, K_COLS };
  int tiles_of(const BInst<T>* I, int kind) const {
    switch (kind) {
      case K_ETILE: return (int)((I->n_el + eb_cur - 1) / eb_cur);
      case K_E256: return I->ntile_e;
      case K_SCHUR: return (int)((I->n_el + kSchurEPB - 1) / kSchurEPB);  // block-Jacobi factor builds
      case K_PREC: return (int)((I->n_el + kPrecEB - 1) / kPrecEB);       // block-Jacobi applies
      case K_VEC: return I->ntile;
      case K_TRACE: return (int)((NFNFC * I->n_el + 255) / 256);
      case K_COLS: return dim == 2 ? (int)I->n_el : cols_tiles_for(BS, (int)I->n_el);  // diagonal-block workgroups
    }
    return 1;
  }
  // fills inst, tile0 and jv (the Krylov index: jv[a] if given, else the
  // instance's current one); rows are zeroed
  int build(BatchSet& S, const std::vector<int>& L, int kind, const std::vector<int>* jv = nullptr) const {
    S.n = (int)L.size();
    int tot = 0;
    for (size_t a = 0; a < L.size(); ++a) {
      const BInst<T>* I = slots[L[a]];
      S.inst[a] = (uint16_t)L[a];
      S.tile0[a] = tot;
      S.jv[a] = (uint8_t)(jv ? (*jv)[a] : I->j);
      S.rows[a] = 0;
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
    return dispatchT<T>(dim, P, f);
  }
  // face traces of slot sX into trL
  int trace(const std::vector<int>& L, int sX) {
    BatchSet S;
    const int nt = build(S, L, K_TRACE);
    if (!nt) return BSW_OK;
    auto f = [&]<int D, int PP, class TT>() -> int {
      hipLaunchKernelGGL((kb_trace<D, PP, TT>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, sX);
      HIPCHK(c, hipGetLastError());
      return BSW_OK;
    };
    ++launches;
    return dispatchT<T>(dim, P, f);
  }
  // The element pass over L (mode 0: residual, 1: Jacobian product) in the
  // tile shape the autotuner picks for this launch's size; t_stop (optional)
  // is recorded by the launch itself when it completes.
  int elem_pass(int mode, const std::vector<int>& L, const std::vector<int>* jv, int sW, int sX, int sOut,
                hipEvent_t t_stop = nullptr, hipEvent_t t_start = nullptr) {
    int64_t n_el = 0;
    for (int k : L) n_el += slots[k]->n_el;
    const uint64_t key = TileTuner::key(dim, P, (int)sizeof(T), mode, n_el);
    bool measure = false;
    const int v = tile_tuner().pick(key, &measure);
    eb_cur = EBv[v];
    BatchSet S;
    const int nt = build(S, L, K_ETILE, jv);
    if (!nt) return BSW_OK;
    hipEvent_t ta = nullptr, tb = nullptr;
    if (measure && (hipEventCreate(&ta) != hipSuccess || hipEventCreate(&tb) != hipSuccess ||
                    hipEventRecord(ta, c->stream) != hipSuccess)) {
      if (ta) (void)hipEventDestroy(ta);
      if (tb) (void)hipEventDestroy(tb);
      ta = tb = nullptr;
    }
    auto f = [&]<int D, int PP, class TT>() -> int {
      auto go = [&]<int V>() {
        if (mode == 0)
          hipExtLaunchKernelGGL((kb_elem<D, PP, TT, 0, V>), dim3(nt), dim3(etile_nt<D, V>()), 0, c->stream,
                                t_start, t_stop, 0, d_desc, S, sW, sX, (int)B_BOLD, sOut);
        else
          hipExtLaunchKernelGGL((kb_elem<D, PP, TT, 1, V>), dim3(nt), dim3(etile_nt<D, V>()), 0, c->stream,
                                t_start, t_stop, 0, d_desc, S, sW, sX, (int)B_BOLD, sOut);
      };
      if (v == 0) go.template operator()<0>();
      else if (v == 1) go.template operator()<1>();
      else go.template operator()<2>();
      HIPCHK(c, hipGetLastError());
      return BSW_OK;
    };
    const int rc = dispatchT<T>(dim, P, f);
    if (ta) {
      if (rc == BSW_OK && hipEventRecord(tb, c->stream) == hipSuccess) {
        tile_tuner().submit(key, v, ta, tb);
      } else {
        (void)hipEventDestroy(ta);
        (void)hipEventDestroy(tb);
      }
    }
    if (rc) return rc;
    ++launches;
    return BSW_OK;
  }
  // mode 0: out = R(W; b_old); mode 1: out = J x (the element pass evaluates
  // the neighbours' side of its argument itself)
  int elem(int mode, const std::vector<int>& L, int sW, int sX, int sOut) {
    return elem_pass(mode, L, nullptr, sW, sX, sOut);
  }
  // traces of the linearisation state for all of L; diagonal blocks and their
  // block-Jacobi factors for the instances in B (a subset of L)
  int linearize(const std::vector<int>& L, const std::vector<int>& B) {
    if (int rc = trace(L, B_W)) return rc;
    BatchSet S;
    const int nt = build(S, B, K_SCHUR);
    if (!nt) return BSW_OK;
    auto f = [&]<int D, int PP, class TT>() -> int {
      BatchSet Sc;
      const int ncol = build(Sc, B, K_COLS);
      if constexpr (D == 2)
        hipLaunchKernelGGL((kb_jac_blocks_tri<PP, TT>), dim3(ncol), dim3(JB2<PP>::NT), 0, c->stream, d_desc, Sc,
                           (int)B_W);
      else
        hipLaunchKernelGGL((kb_jac_columns<D, PP, TT>), dim3(ncol), dim3(256), 0, c->stream, d_desc, Sc, (int)B_W);
      HIPCHK(c, hipGetLastError());
      hipLaunchKernelGGL((kb_schur_build<D, PP, TT>), dim3(nt), dim3(256), 0, c->stream, d_desc, S);
      HIPCHK(c, hipGetLastError());
      return BSW_OK;
    };
    launches += 2;
    return dispatchT<T>(dim, P, f);
  }
  int prec(const std::vector<int>& L, int sX, int sY) {
    BatchSet S;
    const int nt = build(S, L, K_PREC);
    if (!nt) return BSW_OK;
    auto f = [&]<int D, int PP, class TT>() -> int {
      hipLaunchKernelGGL((kb_prec_apply<D, PP, TT>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, sX, sY);
      HIPCHK(c, hipGetLastError());
      return BSW_OK;
    };
    ++launches;
    return dispatchT<T>(dim, P, f);
  }

  // ------------------------------------------------------------ vector stages
  // y = a x + b z (flags as kb_lin); s[] gives the per-instance scalar
  int lin(const std::vector<int>& L, int sy, int sx, int sz, double a, double b, int flags,
          const std::vector<double>* s = nullptr) {
    BatchSetS S;
    const int nt = build(S, L, K_VEC);
    if (!nt) return BSW_OK;
    for (size_t k = 0; k < L.size(); ++k) S.s[k] = s ? (*s)[k] : 0.0;
    hipLaunchKernelGGL((kb_lin<T>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, sy, sx, sz, a, b, flags);
    HIPCHK(c, hipGetLastError());
    ++launches;
    return BSW_OK;
  }
  int combine(const std::vector<int>& L, const std::vector<int>& rows, int coff, int sw, int sy, double sgn,
              int flags, const std::vector<double>* s = nullptr) {
    BatchSetS S;
    const int nt = build(S, L, K_VEC);
    if (!nt) return BSW_OK;
    for (size_t k = 0; k < L.size(); ++k) {
      S.rows[k] = (uint8_t)rows[k];
      S.s[k] = s ? (*s)[k] : 0.0;
    }
    hipLaunchKernelGGL((kb_combine<T>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, (const double*)sc, coff,
                       (int)B_V0, sw, sy, sgn, flags);
    HIPCHK(c, hipGetLastError());
    ++launches;
    return BSW_OK;
  }
  // fold the partials of rows[] rows per instance into sc / sch at offset off
  // (scl, sig, off2: as kb_rows_final; jv: per-instance Krylov index)
  int final_rows(const std::vector<int>& L, const std::vector<int>& rows, int etile, unsigned ops, int off,
                 int scl = 0, int sig = -1, const std::vector<int>* jv = nullptr, int off2 = -1) {
    BatchSet S;
    build(S, L, K_ONE, jv);
    int mr = 0;
    for (size_t k = 0; k < L.size(); ++k) {
      S.rows[k] = (uint8_t)rows[k];
      mr = std::max(mr, rows[k]);
    }
    if (!mr) return BSW_OK;
    hipLaunchKernelGGL((kb_rows_final<T>), dim3((unsigned)L.size(), mr), dim3(256), 0, c->stream, d_desc, S, etile,
                       ops, sc, sch_dev, off, scl, sig, off2);
    HIPCHK(c, hipGetLastError());
    ++launches;
    return BSW_OK;
  }
  // op 0: sum of squares, 1: max |x|, of slot s0 (and s1 >= 0) -> rows 0 (1)
  // at off; sig >= 0 (op 0): the norm is written and sigma_{jv + sig} = 1 / norm;
  // vonly: over the first 1 + D fields only
  int vred(const std::vector<int>& L, int s0, int s1, int op, int off, int sig = -1, int vonly = 0) {
    BatchSet S;
    const int nt = build(S, L, K_VEC);
    if (!nt) return BSW_OK;
    const int nr = s1 >= 0 ? 2 : 1;
    hipLaunchKernelGGL((kb_vred<T>), dim3(nt, nr), dim3(256), 0, c->stream, d_desc, S, s0, s1 >= 0 ? s1 : s0, op,
                       vonly);
    HIPCHK(c, hipGetLastError());
    ++launches;
    std::vector<int> rows(L.size(), nr);
    const unsigned ops = op == 0 ? 0u : (1u | (1u << 2));
    return final_rows(L, rows, 0, ops, off, 0, sig);
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
    if (int rc = dispatchT<T>(dim, P, f)) return rc;
    std::vector<int> rows(L.size(), 4);
    return final_rows(L, rows, 1, 0u | (0u << 2) | (1u << 4) | (2u << 6), kScB);
  }

  // ------------------------------------------------------------ descriptors
  void fill_desc(int k) {
    BInst<T>* I = slots[k];
    InstDesc<T>& d = h_desc[k];
    d.m = view<T>(I->disc);
    bsw_params pc = I->prm;
    if (I->gamma_cur > 0) pc.gamma = I->gamma_cur;
    double v[28];
    dirichlet_table(pc, v);
    for (int i = 0; i < 28; ++i) h_dirtab[(size_t)k * 28 + i] = (T)v[i];
    d.p = devparams<T>(pc, I->dtk > 0 ? I->dtk : I->dt, d_dirtab + (size_t)k * 28);
    d.ws = I->ws;
    d.ld = I->ld;
    d.len = I->len;
    d.len_v = I->len / (1 + dim + dim * dim) * (1 + dim);
    d.blk = (float*)I->disc->blocks;
    d.blk_raw = (T*)I->disc->blocks_raw;
    d.trL = (T*)I->disc->trL;
    d.part = I->part;
    d.ntile = I->ntile;
    d.ntile_e = I->ntile_e;
  }
  // the pinned staging is only rewritten after a stream synchronisation
  int upload_desc() {
    HIPCHK(c, hipMemcpyAsync(d_desc, h_desc, sizeof(InstDesc<T>) * kMaxBatch, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d_dirtab, h_dirtab, sizeof(T) * kMaxBatch * 28, hipMemcpyHostToDevice, c->stream));
    return BSW_OK;
  }

  // ------------------------------------------------------------ admission
  static int64_t part_len(int64_t len, int64_t n_el) {
    return std::max<int64_t>(std::max<int64_t>(130 * ((len + kVT - 1) / kVT), 4 * ((n_el + 255) / 256)), 4096);
  }
  static int64_t ws_len(int64_t len, int M) { return (int64_t)(kBaseSlots + M + 1) * round_up(len, 64); }

  // Puts I in a free slot.  Its workspace and partials are allocated here
  // unless the caller provided them; the initial state comes from W0 (host
  // when w0_dev == 0, device otherwise) or the projection of ic.
  int add(BInst<T>* I, const void* W0, int w0_dev, const bsw_ic* ic) {
    const int k = free_slot();
    if (k < 0) return fail(c, BSW_E_STATE, "batch is full");
    bsw_disc d = I->disc;
    I->n_el = d->mesh->n_el;
    I->len = bsw_state_len(d);
    I->ld = round_up(I->len, 64);
    I->ntile = (int)((I->len + kVT - 1) / kVT);
    I->ntile_e = (int)((I->n_el + 255) / 256);
    const size_t nb = (size_t)BS * BS * I->n_el;
    const size_t nf = (size_t)schur_numbers(dim, n_modes(dim, P)) * I->n_el;
    if (!I->ws && hipMalloc((void**)&I->ws, sizeof(T) * (size_t)ws_len(I->len, M)) != hipSuccess)
      return fail(c, BSW_E_OOM, "instance workspace");
    if ((!d->blocks && hipMalloc(&d->blocks, nf * sizeof(float)) != hipSuccess) ||
        (!d->blocks_raw && hipMalloc(&d->blocks_raw, nb * sizeof(T)) != hipSuccess))
      return fail(c, BSW_E_OOM, "block-Jacobi storage");
    if (!I->part)
      if (int rc = dev_alloc(c, &I->part, (size_t)part_len(I->len, I->n_el))) return rc;
    T* W = I->ws + (size_t)B_W * I->ld;
    if (W0) {
      HIPCHK(c, hipMemcpyAsync(W, W0, sizeof(T) * I->len, w0_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                               c->stream));
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
    I->Hu.assign((size_t)(M + 1) * M, 0.0);
    I->Hp.assign(M + 1, 0.0);
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

  // ------------------------------------------------------------ GMRES (lockstep, pipelined)
  // Right-preconditioned restarted GMRES(M) with classical Gram-Schmidt
  // and delayed reorthogonalisation (kb_gs_dots, kb_gs_update), per
  // instance: J x = rhs to ||rhs - J x|| <= rtol ||rhs|| with x = B_DW
  // starting at 0.  One Arnoldi step of every participating instance is five
  // launches (preconditioner, Jacobian, the pass of dot products, its fold,
  // and the pass that writes the reorthogonalised v_j and the next direction
  // with its norm partials, which the next step's preconditioner pass
  // folds); the Hessenberg column, Givens rotations and the cycle test run
  // on the host from the mapped scalars.  The host issues step t+1 before it
  // reads step t (Krylov index and iteration cap known in advance), so the
  // device never waits on the host; a step issued for an instance whose
  // cycle turned out to end at t is discarded (it only wrote scratch
  // vectors, V_{j+1} and V_{j+2}, which the cycle's solution does not use).
  struct Tick {
    std::vector<int> mem, jv;
    int parity = 0;
  };
  hipEvent_t tick_ev[2] = {nullptr, nullptr};
  hipEvent_t jt0[2] = {nullptr, nullptr}, jt1[2] = {nullptr, nullptr};
  bool timing = false;
  // in timing mode the Jacobian apply of every kTimeEvery-th tick carries
  // HIP events (events on every apply would add their own cost to the solve)
  static constexpr int kTimeEvery = 4;
  int64_t tick_no = 0;
  bool timed_tick[2] = {false, false};
  double jac_seconds = 0.0, jac_launches = 0.0;
  // host time issuing Arnoldi steps and waiting for them (timing mode)
  double issue_seconds = 0.0, wait_seconds = 0.0, arnoldi_steps = 0.0;

  int ensure_events() {
    if (tick_ev[0]) return BSW_OK;
    for (int p = 0; p < 2; ++p) {
      HIPCHK(c, hipEventCreateWithFlags(&tick_ev[p], hipEventDisableTiming));
      HIPCHK(c, hipEventCreate(&jt0[p]));
      HIPCHK(c, hipEventCreate(&jt1[p]));
    }
    return BSW_OK;
  }
  void destroy_events() {
    for (int p = 0; p < 2; ++p) {
      if (tick_ev[p]) (void)hipEventDestroy(tick_ev[p]);
      if (jt0[p]) (void)hipEventDestroy(jt0[p]);
      if (jt1[p]) (void)hipEventDestroy(jt1[p]);
      tick_ev[p] = jt0[p] = jt1[p] = nullptr;
    }
  }

  // The norm of V_{j+1} (from the partials of kb_gs_update) is folded by the
  // next step's preconditioner pass, which needs sigma_{j+1} first; for an
  // instance without a next step, close_norms folds it on its own.  A step's
  // completion event is recorded after those folds.
  int close_norms(const Tick& prev, const std::vector<int>& keep) {
    std::vector<int> L, jv;
    for (size_t a = 0; a < prev.mem.size(); ++a)
      if (std::find(keep.begin(), keep.end(), prev.mem[a]) == keep.end()) {
        L.push_back(prev.mem[a]);
        jv.push_back(prev.jv[a]);
      }
    if (!L.empty()) {
      const std::vector<int> rows(L.size(), 1);
      if (int rc = final_rows(L, rows, 0, 0u, kScN + prev.parity, 0, 1, &jv)) return rc;
    }
    HIPCHK(c, hipEventRecord(tick_ev[prev.parity], c->stream));
    return BSW_OK;
  }

  // one pipelined Arnoldi step of the instances in tk; prev: the step issued
  // before it (its norms are folded here), or null
  int launch_tick(const Tick& tk, const Tick* prev) {
    const std::vector<int>& L = tk.mem;
    const std::vector<int>* jv = &tk.jv;
    const int pa = tk.parity;
    const int offA = pa ? kScA1 : kScA, offB = pa ? kScB1 : kScB;
    const bool tm = timing && tick_no++ % kTimeEvery == 0;
    timed_tick[pa] = tm;
    BatchSet S;
    // z = sigma_j M^{-1} V_j, sigma_j folded here for instances continuing prev
    int nt = build(S, L, K_PREC, jv);
    for (size_t a = 0; a < L.size(); ++a)
      S.rows[a] = prev && std::find(prev->mem.begin(), prev->mem.end(), L[a]) != prev->mem.end() ? 1 : 0;
    const int offN = kScN + (prev ? prev->parity : 0);
    auto fp = [&]<int D, int PP, class TT>() -> int {
      hipLaunchKernelGGL((kb_prec_krylov<D, PP, TT>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, sc, sch_dev,
                         offN, (int)B_V0, (int)B_Z);
      HIPCHK(c, hipGetLastError());
      return BSW_OK;
    };
    if (int rc = dispatchT<T>(dim, P, fp)) return rc;
    if (prev)
      if (int rc = close_norms(*prev, L)) return rc;
    // w = J z: one element pass (the neighbours' side of z evaluated in it)
    if (int rc = elem_pass(1, L, jv, (int)B_W, (int)B_Z, (int)B_WK, tm ? jt1[pa] : nullptr, tm ? jt0[pa] : nullptr))
      return rc;
    --launches;  // counted with the tick's own launches below
    // pass 1: V^T y_j, V^T w with y_j . y_j and y_j . w (row pairs)
    nt = build(S, L, K_VEC, jv);
    int maxrows = 0;
    for (int j : tk.jv) maxrows = std::max(maxrows, j + 1);
    if (maxrows <= kRowsCached)
      hipLaunchKernelGGL((kb_gs_dots_cached<T>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, (int)B_V0, (int)B_WK);
    else
      hipLaunchKernelGGL((kb_gs_dots<T>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, (int)B_V0, (int)B_WK);
    HIPCHK(c, hipGetLastError());
    std::vector<int> rows(L.size());
    for (size_t a = 0; a < L.size(); ++a) rows[a] = 2 * (tk.jv[a] + 1);
    if (int rc = final_rows(L, rows, 0, 0u, offA, 1, -1, jv, offB)) return rc;
    // pass 2: v_j final in place, u_{j+1} -> V_{j+1} with its norm partials
    hipLaunchKernelGGL((kb_gs_update<T>), dim3(nt), dim3(256), 0, c->stream, d_desc, S, sc, sch_dev, offA, offB,
                       kScN + 6 + pa, kScN + 8 + pa, (int)B_V0, (int)B_WK);
    HIPCHK(c, hipGetLastError());
    launches += 4;  // prec, element pass, two Gram-Schmidt passes (folds count themselves)
    return BSW_OK;
  }

  // Step j of one instance from its scalars: completes Hessenberg column
  // j - 1 (its Arnoldi relation took u_j = ||u_j|| y_j, and y_j = V s +
  // rho v_j), rotates it, then forms column j from this step's t and c
  // against the completed columns (h_kj = (t_k - (Hu s)_k) / rho, the last
  // entry ||u_{j+1}||), rotates a copy for the residual estimate and the
  // cycle test.  Column j stays open until the next step completes it; a
  // cycle that ends here solves with it as it stands (the true residual is
  // formed at the cycle end).
  void arnoldi_update(BInst<T>* I, int k, int j, int pa) {
    const int offA = pa ? kScA1 : kScA, offB = pa ? kScB1 : kScB;
    double* H = I->H.data();
    double* Hu = I->Hu.data();
    double* cs = I->cs.data();
    double* sn = I->sn.data();
    double* g = I->g.data();
    const double rho = rd(k, kScN + 6 + pa), cc = rd(k, kScN + 8 + pa);
    const double rn = rd(k, kScN + pa);  // ||u_{j+1}||
    auto rotate = [&](double* col, int upto) {
      for (int i = 0; i < upto; ++i) {
        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
      }
    };
    auto close = [&](double* col, int jc) {  // rotation jc from col[jc], col[jc + 1]
      const double den = std::hypot(col[jc], col[jc + 1]);
      cs[jc] = den > 0.0 ? col[jc] / den : 1.0;
      sn[jc] = den > 0.0 ? col[jc + 1] / den : 0.0;
      col[jc] = den;
      col[jc + 1] = 0.0;
      for (int i = 0; i <= jc + 1; ++i) H[(size_t)i * M + jc] = col[i];
      g[jc + 1] = -sn[jc] * g[jc];
      g[jc] = cs[jc] * g[jc];
    };
    double col[66];
    if (j >= 1) {
      const double r = I->hn;  // ||u_j||
      for (int i = 0; i < j; ++i) col[i] = I->Hp[i] + r * rd(k, offA + i);
      col[j] = r * rho;
      for (int i = 0; i <= j; ++i) Hu[(size_t)i * M + j - 1] = col[i];
      rotate(col, j - 1);
      g[j - 1] = I->gsave;
      close(col, j - 1);
    }
    const double rinv = rho > 0.0 ? 1.0 / rho : 0.0;
    for (int kk = 0; kk <= j; ++kk) {
      double hs = 0.0;
      for (int i = std::max(0, kk - 1); i < j; ++i) hs += Hu[(size_t)kk * M + i] * rd(k, offA + i);
      const double tk = kk < j ? rd(k, offB + kk) : cc;
      col[kk] = (tk - hs) * rinv;
      I->Hp[kk] = col[kk];
    }
    col[j + 1] = rn;
    rotate(col, j);
    I->gsave = g[j];
    close(col, j);
    I->hn = rn;
    I->cyc_conv = std::fabs(g[j + 1]) <= I->rtol * I->bn || rn == 0.0;
    I->iters += 1;
    I->j = j + 1;
  }

  // cycle end of the instances in E: x += M^{-1} V y, true residual
  // rhs - J x -> V_0 (sigma_0 = 1 / its norm); returns after the norms are read
  int cycle_end(const std::vector<int>& E) {
    std::vector<int> rows;
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
      HIPCHK(c, hipMemcpyAsync(sc + (size_t)k * kScStride + kScY, st, sizeof(double) * jj, hipMemcpyHostToDevice,
                               c->stream));
      rows.push_back(jj);
      I->cycles += 1;
    }
    if (int rc = combine(E, rows, kScY, B_WK, B_Z, 1.0, 2 | 8)) return rc;
    if (int rc = prec(E, B_Z, B_U)) return rc;
    if (int rc = lin(E, B_DW, B_DW, B_U, 1.0, 1.0, 0)) return rc;
    if (int rc = elem(1, E, B_W, B_DW, B_WK)) return rc;
    if (int rc = lin(E, B_V0, B_RHS, B_WK, 1.0, -1.0, 0)) return rc;
    std::vector<int> zero(E.size(), 0);
    for (int k : E) slots[k]->j = 0;  // sigma_0 is written at jv + 0
    if (int rc = vred(E, B_V0, -1, 0, kScN + 3, 0)) return rc;
    return sync();
  }

  int gmres(const std::vector<int>& N) {
    if (int rc = ensure_events()) return rc;
    if (int rc = lin(N, B_DW, B_DW, B_DW, 0.0, 0.0, 4)) return rc;
    if (int rc = lin(N, B_V0, B_RHS, B_RHS, 1.0, 0.0, 8)) return rc;
    for (int k : N) slots[k]->j = 0;
    if (int rc = vred(N, B_V0, -1, 0, kScN + 2, 0)) return rc;
    if (int rc = sync()) return rc;
    Tick cur, nxt;
    int parity = 0;
    for (int k : N) {
      BInst<T>* I = slots[k];
      I->iters = 0;
      I->cycles = 0;
      I->relres = 0.0;
      I->bn = rd(k, kScN + 2);
      I->beta = I->bn;
      I->j = 0;
      if (I->bn > 0.0) {
        std::fill(I->g.begin(), I->g.end(), 0.0);
        I->g[0] = I->bn;
        cur.mem.push_back(k);
        cur.jv.push_back(0);
      }
    }
    cur.parity = parity;
    if (!cur.mem.empty())
      if (int rc = launch_tick(cur, nullptr)) return rc;
    std::vector<int> rejoin, E;
    std::vector<char> dropped(kMaxBatch, 0);
    while (!cur.mem.empty() || !rejoin.empty()) {
      // issue the next step ahead of reading this one
      nxt.mem.clear();
      nxt.jv.clear();
      nxt.parity = 1 - cur.parity;
      for (size_t a = 0; a < cur.mem.size(); ++a) {
        const BInst<T>* I = slots[cur.mem[a]];
        if (cur.jv[a] + 2 <= M && I->iters + 2 <= I->opt.gmres_max_iters) {
          nxt.mem.push_back(cur.mem[a]);
          nxt.jv.push_back(cur.jv[a] + 1);
        }
      }
      for (int k : rejoin) {
        nxt.mem.push_back(k);
        nxt.jv.push_back(0);
      }
      rejoin.clear();
      if (!nxt.mem.empty()) {
        // keep engine-slot order (instance order inside launches)
        std::vector<size_t> ord(nxt.mem.size());
        for (size_t a = 0; a < ord.size(); ++a) ord[a] = a;
        std::sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return nxt.mem[x] < nxt.mem[y]; });
        Tick sorted;
        sorted.parity = nxt.parity;
        for (size_t a : ord) {
          sorted.mem.push_back(nxt.mem[a]);
          sorted.jv.push_back(nxt.jv[a]);
        }
        nxt = sorted;
        const auto h0 = std::chrono::steady_clock::now();
        if (int rc = launch_tick(nxt, cur.mem.empty() ? nullptr : &cur)) return rc;
        if (timing) issue_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - h0).count();
      } else if (!cur.mem.empty()) {
        if (int rc = close_norms(cur, {})) return rc;
      }
      if (!cur.mem.empty()) {
        const auto h0 = std::chrono::steady_clock::now();
        HIPCHK(c, hipEventSynchronize(tick_ev[cur.parity]));
        if (timing) {
          wait_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - h0).count();
          arnoldi_steps += 1;
        }
        ++ticks;
        if (timing && timed_tick[cur.parity]) {
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, jt0[cur.parity], jt1[cur.parity]) == hipSuccess) {
            jac_seconds += 1e-3 * ms;
            jac_launches += 1;
          }
        }
        E.clear();
        for (size_t a = 0; a < cur.mem.size(); ++a) {
          const int k = cur.mem[a];
          BInst<T>* I = slots[k];
          arnoldi_update(I, k, cur.jv[a], cur.parity);
          if (I->cyc_conv || I->j == M || I->iters >= I->opt.gmres_max_iters) E.push_back(k);
        }
        if (!E.empty()) {
          for (int k : E) dropped[k] = 1;
          if (int rc = cycle_end(E)) return rc;
          for (int k : E) {
            BInst<T>* I = slots[k];
            I->beta = rd(k, kScN + 3);
            I->relres = I->beta / I->bn;
            if (I->cyc_conv || I->beta <= I->rtol * I->bn || I->iters >= I->opt.gmres_max_iters) continue;
            I->j = 0;
            std::fill(I->g.begin(), I->g.end(), 0.0);
            I->g[0] = I->beta;
            rejoin.push_back(k);
          }
        }
      }
      // the issued step of an instance whose cycle ended is discarded
      cur.mem.clear();
      cur.jv.clear();
      cur.parity = nxt.parity;
      for (size_t a = 0; a < nxt.mem.size(); ++a)
        if (!dropped[nxt.mem[a]]) {
          cur.mem.push_back(nxt.mem[a]);
          cur.jv.push_back(nxt.jv[a]);
        }
      std::fill(dropped.begin(), dropped.end(), 0);
    }
    return BSW_OK;
  }

  // ------------------------------------------------------------ one time step
  int step_all() {
    std::vector<int> S;
    for (int k = 0; k < kMaxBatch; ++k)
      if (slots[k] && !slots[k]->finished()) S.push_back(k);
    if (S.empty()) return BSW_OK;
    // continuation stages (one unless requested), each a Newton solve from the
    // last; gamma of stage i (0-based) of n: gamma0 + i (gamma - gamma0) / (n - 1)
    auto stage_gamma = [](const BInst<T>* I, int stg) {
      return I->nstage >= 2 ? I->opt.cont_gamma0 + stg * (I->prm.gamma - I->opt.cont_gamma0) / (I->nstage - 1) : 0.0;
    };
    for (int k : S) {
      BInst<T>* I = slots[k];
      const int kk = I->step + 1;
      I->dtk = kk < I->n_total ? I->dt : I->opt.t_end - (kk - 1) * I->dt;
      I->nstage = I->opt.cont_steps >= 2 ? I->opt.cont_steps : 1;
      I->stage = 0;
      I->it_step = 0;
      I->conv = 0;
      I->gamma_cur = stage_gamma(I, 0);
      fill_desc(k);
    }
    if (int rc = upload_desc()) return rc;
    if (int rc = step_begin(S)) return rc;
    // ||b_old|| for the residual stopping test (res_tol)
    std::vector<int> Sr;
    for (int k : S)
      if (res_tol_of(slots[k]) > 0) Sr.push_back(k);
    if (!Sr.empty()) {
      if (int rc = vred(Sr, B_BOLD, -1, 0, kScN + 4, -1, 1)) return rc;
      if (int rc = sync()) return rc;
      for (int k : Sr) slots[k]->bold_norm = std::sqrt(rd(k, kScN + 4));
    }
    for (int stg = 0;; ++stg) {
      std::vector<int> Sg;
      for (int k : S) {
        BInst<T>* I = slots[k];
        if (stg >= I->nstage || I->conv < 0) continue;
        Sg.push_back(k);
      }
      if (Sg.empty()) break;
      if (stg > 0) {
        // the previous stage ended with a stream synchronisation: the staging
        // copy of the descriptors has completed and may be rewritten
        for (int k : Sg) {
          BInst<T>* I = slots[k];
          I->stage = stg;
          I->gamma_cur = stage_gamma(I, stg);
          fill_desc(k);
        }
        if (int rc = upload_desc()) return rc;
      }
      if (int rc = newton(Sg)) return rc;
    }
    for (int k : S) {
      slots[k]->gamma_cur = 0.0;
      fill_desc(k);
    }
    if (int rc = upload_desc()) return rc;
    if (int rc = diag(S)) return rc;
    if (int rc = sync()) return rc;
    for (int k : S) {
      BInst<T>* I = slots[k];
      I->st.newton_total += I->it_step;
      I->st.newton_max = std::max(I->st.newton_max, I->it_step);
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

  // residual stopping test: ||R||_2 <= res_tol ||b_old||_2 (res_tol 0 selects
  // 1e-13, a negative value turns it off)
  static double res_tol_of(const BInst<T>* I) { return I->opt.res_tol == 0 ? 1e-13 : I->opt.res_tol; }
  static bool res_converged(const BInst<T>* I) {
    const double rt = res_tol_of(I);
    return rt > 0 && std::isfinite(I->rn) && I->rn <= rt * I->bold_norm;
  }

  // Newton for the instances in S at the parameters in their descriptors:
  // residual, then up to max_newton iterations of linearise, GMRES, update test
  // and backtracking; it_step accumulates the iterations, conv the outcome
  int newton(const std::vector<int>& S) {
    if (int rc = elem(0, S, B_W, B_W, B_R)) return rc;
    if (int rc = vred(S, B_R, -1, 0, kScB)) return rc;
    if (int rc = sync()) return rc;
    for (int k : S) {
      BInst<T>* I = slots[k];
      I->st.operator_applies += 1;
      I->rn = std::sqrt(rd(k, kScB));
      I->rn_prev = I->rn;
      I->it = 0;
      I->conv = res_converged(I) ? 1 : 0;
      I->eta = I->opt.forcing_max > 0 ? I->opt.forcing_max : 3e-2;
    }
    std::vector<int> N, C, L, A, nxt;
    for (int k : S)
      if (slots[k]->conv == 0) N.push_back(k);
    std::vector<double> s;
    while (!N.empty()) {
      for (int k : N) {
        BInst<T>* I = slots[k];
        I->it += 1;
        // Eisenstat-Walker forcing (choice 2, gamma 0.9, exponent 2) in [gmres_rtol, forcing_max]
        if (I->it > 1) {
          const double r = I->rn / std::max(I->rn_prev, 1e-300);
          const double cand = 0.9 * r * r, safe = 0.9 * I->eta * I->eta;
          I->eta = std::max(cand, safe > 0.1 ? safe : 0.0);
        }
        I->eta = std::min(I->opt.forcing_max > 0 ? I->opt.forcing_max : 3e-2, std::max(I->eta, I->gmres_rtol));
        I->rtol = I->eta;
      }
      // the block-Jacobi preconditioner is rebuilt every Newton iteration; with
      // precond_lag it is built at the first iteration of a Newton solve and
      // kept while it still serves: rebuilt when the last GMRES solve missed
      // its tolerance or took more than 1.5x (+10) the iterations of the first
      // solve after the last build
      std::vector<int> Bk;
      for (int k : N) {
        BInst<T>* I = slots[k];
        const bool stale = !I->gm_ok || I->gm_last > 1.5 * I->gm_ref + 10;
        I->rebuilt = I->opt.precond_lag <= 0 || I->it == 1 || stale;
        if (I->rebuilt) Bk.push_back(k);
      }
      if (int rc = linearize(N, Bk)) return rc;
      if (int rc = lin(N, B_RHS, B_R, B_R, -1.0, 0.0, 8)) return rc;
      if (int rc = gmres(N)) return rc;
      for (int k : N) {
        BInst<T>* I = slots[k];
        I->st.gmres_total += I->iters;
        I->st.jacobian_applies += I->iters + I->cycles;
        I->gm_last = I->iters;
        I->gm_ok = I->relres <= 10.0 * I->rtol;
        if (I->rebuilt) I->gm_ref = I->iters;
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
          else if (res_converged(I)) I->conv = 1;
        }
        L = nxt;
      }
      nxt.clear();
      for (int k : N)
        if (slots[k]->conv == 0 && slots[k]->it < slots[k]->opt.max_newton) nxt.push_back(k);
      N = nxt;
    }
    for (int k : S) slots[k]->it_step += slots[k]->it;
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
  bsw_bed bed{};
  int orders[3] = {-1, -1, -1};  // m1, m2, m3 (-1: the uniform order P)
  std::vector<int8_t> face_bc;    // per-face boundary codes (empty: the parameters' bc)
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
    if (!rc && !r->face_bc.empty()) rc = bsw_mesh_set_boundary(I->mesh, r->face_bc.data());
    if (!rc) rc = bsw_disc_create(I->mesh, r->P, r->precision, &I->disc);
    if (!rc) rc = check_params(I->disc, &I->prm);
    if (!rc && r->orders[0] >= 0) rc = bsw_disc_set_orders(I->disc, r->orders[0], r->orders[1], r->orders[2]);
    if (!rc && r->bed.kind != BSW_BED_FLAT) {
      if (hipMalloc((void**)&I->bed, sizeof(T) * (size_t)n_modes(2, r->P) * r->n_el) != hipSuccess)
        rc = fail(c, BSW_E_OOM, "bed coefficients");
      if (!rc) rc = bsw_bed_interpolate(I->disc, &r->bed, I->bed);
      if (!rc) rc = bsw_disc_set_bed(I->disc, I->bed);
    }
    if (!rc) rc = e.add(I, r->W0.empty() ? nullptr : r->W0.data(), 0, &r->ic);
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

// One worker thread and one HIP stream per engine, so the batches of different
// (order, precision, restart length) run concurrently on the device and a
// slow batch does not hold up the others.
struct EngineRec {
  long key = 0;
  bsw_ctx_s ctx;  // the engine's own context and stream
  std::unique_ptr<EngineIf> eng;
  std::thread th;
};

struct bsw_server_s {
  bsw_ctx user = nullptr;
  int device = 0;
  size_t budget = 0;
  int max_slots = 0;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<Request*> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::map<long, std::unique_ptr<EngineRec>> engines;  // key: (P, precision, M)
  uint64_t next_ticket = 1;
  int64_t in_use = 0;
  int resident = 0, peak_resident = 0;
  int64_t steps = 0, completed = 0;
  bool stop = false;

  static long key(const Request* r) { return ((long)r->P * 4 + r->precision) * 256 + r->M; }

  // under mu: the engine of r's key, created with its worker on first use
  int ensure_engine(const Request* r, std::string& err) {
    if (engines.count(key(r))) return BSW_OK;
    auto rec = std::make_unique<EngineRec>();
    rec->key = key(r);
    rec->ctx.device = device;
    if (hipStreamCreateWithFlags(&rec->ctx.stream, hipStreamNonBlocking) != hipSuccess) {
      err = "hipStreamCreateWithFlags";
      return BSW_E_HIP;
    }
    int rc;
    if (r->precision == BSW_FP64) {
      auto* x = new EngineImpl<double>();
      rec->eng.reset(x);
      rc = x->e.init(&rec->ctx, 2, r->P, r->M);
    } else {
      auto* x = new EngineImpl<float>();
      rec->eng.reset(x);
      rc = x->e.init(&rec->ctx, 2, r->P, r->M);
    }
    if (rc) {
      err = rec->ctx.err;
      rec->eng.reset();
      (void)hipStreamDestroy(rec->ctx.stream);
      return rc;
    }
    EngineRec* p = rec.get();
    engines[rec->key] = std::move(rec);
    p->th = std::thread([this, p] { worker(p); });
    return BSW_OK;
  }

  void finish(Request* r) {  // under mu
    r->t_end = std::chrono::steady_clock::now();
    r->st.queue_seconds = std::chrono::duration<double>(r->t_start - r->t_submit).count();
    r->st.seconds = std::chrono::duration<double>(r->t_end - r->t_start).count();
    in_use -= r->footprint;
    resident -= 1;
    completed += 1;
  }

  // Between time steps: drop cancelled queued requests of this engine, admit
  // its queued requests in FIFO order while the footprint fits the budget and
  // a slot is free, step the batch, retire finished solves.
  void worker(EngineRec* rec) {
    (void)hipSetDevice(device);
    EngineIf* E = rec->eng.get();
    std::vector<Request*> adm, out;
    for (;;) {
      adm.clear();
      {
        std::unique_lock<std::mutex> lk(mu);
        if (stop) break;
        int free_slots = kMaxBatch - E->resident();
        for (auto it = queue.begin(); it != queue.end();) {
          Request* r = *it;
          if (key(r) != rec->key) {
            ++it;
            continue;
          }
          if (r->cancel.load()) {
            r->state = BSW_REQ_CANCELLED;
            it = queue.erase(it);
            cv_done.notify_all();
            continue;
          }
          if (resident >= max_slots || in_use + r->footprint > (int64_t)budget || free_slots <= 0) break;
          it = queue.erase(it);
          resident += 1;
          free_slots -= 1;
          in_use += r->footprint;
          peak_resident = std::max(peak_resident, resident);
          r->t_start = std::chrono::steady_clock::now();
          r->state = BSW_REQ_RUNNING;
          adm.push_back(r);
        }
        if (adm.empty() && E->resident() == 0) {
          cv.wait_for(lk, std::chrono::milliseconds(20));
          continue;
        }
      }
      for (Request* r : adm) {
        std::string err;
        const int rc = E->admit(r, err);
        if (rc) {
          std::lock_guard<std::mutex> lk(mu);
          r->rc = rc;
          r->err = err;
          finish(r);
          completed -= 1;
          r->state = BSW_REQ_FAILED;
          cv_done.notify_all();
          cv.notify_all();
        }
      }
      if (!E->resident()) continue;
      out.clear();
      const int rc = E->step();
      if (rc < 0) {
        const std::string err = rec->ctx.err;
        E->drop_all(out);
        std::lock_guard<std::mutex> lk(mu);
        for (Request* r : out) {
          r->rc = rc;
          r->err = err;
          finish(r);
          r->state = BSW_REQ_FAILED;
        }
        cv_done.notify_all();
        cv.notify_all();
        continue;
      }
      E->retire(out);
      std::lock_guard<std::mutex> lk(mu);
      steps += 1;
      for (Request* r : out) {
        finish(r);
        r->state = r->next_state;
      }
      if (!out.empty()) {
        cv_done.notify_all();
        cv.notify_all();  // budget and slots freed: other engines may admit
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
  if (o.cont_steps >= 2 && !(o.cont_gamma0 > 0)) return fail(c, BSW_E_ARG, "continuation needs cont_gamma0 > 0");
  const bsw_params* p = &q->params;
  if (p->reg < 1 || p->reg > 3 || p->bc < 1 || p->bc > 3) return fail(c, BSW_E_ARG, "bad reg or bc");
  if (!(p->g > 0) || !(p->rho > 0) || p->eta < 0 || p->sigma0 < 0 || !(p->gamma > 0) || !(p->beta > 0))
    return fail(c, BSW_E_ARG, "need g, rho, gamma, beta > 0 and eta, sigma0 >= 0");
  if (p->reg != 3 && p->sigma0 > 0 && p->sigma0 < 0.5 / p->beta)
    return fail(c, BSW_E_ARG, "regularisations 1 and 2 need sigma0 >= 1/(2 beta)");
  const bsw_bed& b = q->bed;
  if (b.kind < BSW_BED_FLAT || b.kind > BSW_BED_GAUSS || (b.kind != BSW_BED_FLAT && (b.order < 0 || b.order > q->P)) ||
      (b.kind == BSW_BED_GAUSS && !(b.d > 0)))
    return fail(c, BSW_E_ARG, "bad bed (kind, order 0..P, GAUSS d > 0)");
  if (q->face_bc)
    for (int64_t k = 0; k < 3 * q->n_el; ++k)
      if (q->face_bc[k] < 0 || q->face_bc[k] > 15) return fail(c, BSW_E_ARG, "boundary codes must be in 0..15");
  if (q->mixed_orders) {
    const int m[3] = {q->m1, q->m2, q->m3};
    for (int k = 0; k < 3; ++k)
      if (m[k] < 0 || m[k] > q->P) return fail(c, BSW_E_ARG, "orders m1, m2, m3 must be in 0..P");
  }
  return BSW_OK;
}
}  // namespace

extern "C" {

int bsw_tile_policy(int policy, int* previous) {
  if (policy < -1 || policy >= kTileShapes) return fail(nullptr, BSW_E_ARG, "tile policy must be -1, 0, 1 or 2");
  TileTuner& t = tile_tuner();
  std::lock_guard<std::mutex> lk(t.mu);
  if (previous) *previous = t.policy;
  t.policy = policy;
  return BSW_OK;
}

int bsw_tile_table(double* rows, int max_rows, int* n_rows) {
  if (!n_rows || (max_rows > 0 && !rows)) return fail(nullptr, BSW_E_ARG, "null argument");
  TileTuner& t = tile_tuner();
  std::lock_guard<std::mutex> lk(t.mu);
  t.poll_locked();
  int n = 0;
  for (const auto& kv : t.tab) {
    if (n < max_rows) {
      const uint64_t k = kv.first;
      const TileTuner::Entry& E = kv.second;
      double* r = rows + (size_t)n * 10;
      r[0] = (double)(k & 15);
      r[1] = (double)((k >> 4) & 15);
      r[2] = (double)((k >> 8) & 255);
      r[3] = (double)((k >> 16) & 255);
      r[4] = (double)((k >> 24) & 255);
      r[5] = (double)E.choice;
      for (int v = 0; v < kTileShapes; ++v) r[6 + v] = E.n[v] ? 1e3 * E.best_ms[v] : -1.0;
      r[9] = (double)(E.n[0] + E.n[1] + E.n[2]);
    }
    ++n;
  }
  *n_rows = n;
  return BSW_OK;
}

int64_t bsw_request_footprint(const bsw_solve_request* q) {
  if (!q || q->P < 1 || q->P > 3 || q->n_el < 1) return -1;
  return instance_bytes(q->n_el, 2, q->P, q->precision, std::max(1, std::min(64, q->opts.gmres_m)));
}

int bsw_server_create(bsw_ctx ctx, size_t hbm_budget_bytes, int max_slots, bsw_server* out) {
  if (!ctx || !out) return fail(ctx, BSW_E_ARG, "null argument");
  if (max_slots < 1 || hbm_budget_bytes == 0) return fail(ctx, BSW_E_ARG, "need max_slots >= 1 and a budget");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  auto* S = new bsw_server_s();
  S->user = ctx;
  S->device = ctx->device;
  S->budget = hbm_budget_bytes;
  S->max_slots = max_slots;
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
  for (auto& kv : S->engines)
    if (kv.second->th.joinable()) kv.second->th.join();
  (void)hipSetDevice(S->device);
  for (auto& kv : S->engines) {
    (void)hipStreamSynchronize(kv.second->ctx.stream);
    kv.second->eng.reset();
    (void)hipStreamDestroy(kv.second->ctx.stream);
  }
  S->engines.clear();
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
    const size_t bytes = (size_t)7 * n_modes(2, q->P) * q->n_el * (q->precision == BSW_FP64 ? 8 : 4);
    r->W0.assign((const unsigned char*)q->W0, (const unsigned char*)q->W0 + bytes);
  }
  r->prm = q->params;
  r->ic = q->ic;
  r->bed = q->bed;
  if (q->face_bc) r->face_bc.assign(q->face_bc, q->face_bc + 3 * q->n_el);
  if (q->mixed_orders) {
    r->orders[0] = q->m1;
    r->orders[1] = q->m2;
    r->orders[2] = q->m3;
  }
  r->opt = q->opts;
  r->footprint = bsw_request_footprint(q);
  if (r->footprint > (int64_t)S->budget) return fail(S->user, BSW_E_ARG, "request footprint exceeds the server budget");
  r->t_submit = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    std::string err;
    if (int rc = S->ensure_engine(r.get(), err)) return fail(S->user, rc, "batch engine: " + err);
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
  for (auto& kv : S->engines) launches += kv.second->eng->launches();
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

// ====================================================================== whole solve of one discretisation
namespace {

// bsw_solve: the batch engine with one borrowed instance.  The engine, the
// Krylov workspace and the reduction partials stay cached on the
// discretisation between calls.
template <class T>
int solve_one(bsw_disc d, const bsw_params* p, const bsw_solve_opts* o, T* W, bsw_solve_stats* st) {
  bsw_ctx c = d->mesh->ctx;
  const int M = std::max(1, std::min(64, o->gmres_m));
  auto* E = static_cast<EngineImpl<T>*>(d->eng);
  if (!E || E->e.M != M) {
    if (d->eng) d->eng_free(d->eng);
    d->eng = nullptr;
    E = new EngineImpl<T>();
    if (int rc = E->e.init(c, d->mesh->dim, d->P, M)) {
      delete E;
      return rc;
    }
    d->eng = E;
    d->eng_free = [](void* x) { delete static_cast<EngineImpl<T>*>(x); };
  }
  const int64_t len = bsw_state_len(d);
  const size_t need = sizeof(T) * (size_t)BatchEngine<T>::ws_len(len, M);
  if (d->gm_bytes < need) {
    hfree(d->gm);
    d->gm = nullptr;
    d->gm_bytes = 0;
    if (hipMalloc(&d->gm, need) != hipSuccess) return fail(c, BSW_E_OOM, "solver workspace");
    d->gm_bytes = need;
  }
  if (int rc = ensure_part(d, (size_t)BatchEngine<T>::part_len(len, d->mesh->n_el))) return rc;
  auto t0 = std::chrono::steady_clock::now();
  std::memset(st, 0, sizeof(*st));
  BInst<T>* I = new BInst<T>();
  I->own = false;
  I->mesh = d->mesh;
  I->disc = d;
  I->ws = (T*)d->gm;
  I->part = d->part;
  I->prm = *p;
  I->opt = *o;
  if (int rc = E->e.add(I, W, 1, nullptr)) {
    delete I;
    return rc;
  }
  E->e.timing = o->timing != 0;
  E->e.jac_seconds = 0.0;
  E->e.jac_launches = 0.0;
  E->e.issue_seconds = E->e.wait_seconds = E->e.arnoldi_steps = 0.0;
  int rc = BSW_OK;
  while (!I->finished())
    if ((rc = E->e.step_all())) break;
  if (!rc) {
    hipError_t he = hipMemcpyAsync(W, I->ws + (size_t)B_W * I->ld, sizeof(T) * I->len, hipMemcpyDeviceToDevice,
                                   c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) rc = fail(c, BSW_E_HIP, std::string("state copy: ") + hipGetErrorString(he));
  }
  E->e.final_stats(I);
  *st = I->st;
  st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  st->jac_apply_seconds = E->e.jac_seconds;
  st->jac_apply_launches = E->e.jac_launches;
  st->host_issue_seconds = E->e.issue_seconds;
  st->host_wait_seconds = E->e.wait_seconds;
  st->arnoldi_steps = E->e.arnoldi_steps;
  E->e.take(I->slot);
  delete I;
  return rc ? rc : st->status;
}

}  // namespace

extern "C" int bsw_solve(bsw_disc d, const bsw_params* p, const bsw_solve_opts* o, void* W, bsw_solve_stats* st) {
  if (!d || !o || !W || !st) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "null argument");
  if (int rc = check_params(d, p)) return rc;
  if (o->max_newton < 1 || o->gmres_max_iters < 1 || !(o->t_end > 0))
    return fail(d->mesh->ctx, BSW_E_ARG, "bad solve options");
  if (!(o->dt > 0) && !(o->cfl > 0)) return fail(d->mesh->ctx, BSW_E_ARG, "need dt > 0 or cfl > 0");
  if (o->cont_steps >= 2 && !(o->cont_gamma0 > 0))
    return fail(d->mesh->ctx, BSW_E_ARG, "continuation needs cont_gamma0 > 0");
  if (d->precision == BSW_FP64) return solve_one<double>(d, p, o, (double*)W, st);
  return solve_one<float>(d, p, o, (float*)W, st);
}

