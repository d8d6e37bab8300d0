// Host side of the library: C ABI (include/bsw.h), mesh and discretisation
// setup, kernel dispatch over (dimension, order, precision), deterministic
// reductions, and the backward-Euler / Newton / block-Jacobi GMRES driver.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/bsw.h"
#include "bsw_elem2.hpp"
#include "ref_element.hpp"

namespace bsw {
__constant__ __align__(16) unsigned char c_tables[kTabBytesTotal];
}

// Reduction scratch of the entry points that allocate nothing
// (bsw_stage_update_noalloc): up to kScratchPartials per-workgroup partial
// sums and kScratchOut final values.  Each device the library runs on holds
// one copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the device (bsw_ctx_s::scratch).
constexpr int kScratchPartials = 4 * 1024;
constexpr int kScratchOut = 64;
static __device__ __align__(256) double scratch[kScratchPartials + kScratchOut];
constexpr int kMaxScratchDevices = 64;
static double* g_scratch_dev[kMaxScratchDevices] = {};  // per device: its scratch address
static std::mutex g_scratch_mu;

using namespace bsw;

// ====================================================================== handles
struct bsw_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool tables_staged[2][kNumCombos] = {};
  double* scratch = nullptr;  // this device's copy of the file-scope scratch array
};

template <class T>
struct DevMesh {
  T* dxi = nullptr;
  T* detJ = nullptr;
  T* nrm = nullptr;
  T* hlen = nullptr;
};

struct bsw_mesh_s {
  bsw_ctx ctx = nullptr;
  int dim = 0, nfc = 0;
  int64_t n_el = 0, n_vert = 0;
  double hmin = 0.0, measure = 0.0;
  int* nbr = nullptr;      // device [nfc][n_el]
  double* vert = nullptr;  // device [(dim+1)*dim][n_el]
  DevMesh<double> m64;
  DevMesh<float> m32;
  std::vector<double> h_dxi, h_detJ, h_nrm, h_hlen;  // host copies for the FP32 view
  std::vector<int> h_nbr;                            // host copy of the face map (boundary: -1)
};

struct bsw_disc_s {
  bsw_mesh mesh = nullptr;
  int P = 0, precision = BSW_FP64;
  RefElement ref;
  int bs = 0;
  size_t wsize = 0;  // bytes per real
  const void* bed = nullptr;   // bed coefficients [n_p][n_el] (caller's device memory), nullptr = flat
  void* dirtab = nullptr;      // device [4][7]: Dirichlet states of boundary tags 0..3
  double dirtab_host[28] = {}; // the values last written there
  bool dirtab_set = false;
  int nmode[3] = {0, 0, 0};    // modes used by h, u and E (orders m1, m2, m3)
  // linearisation
  const void* lin_W = nullptr;
  bsw_params lin_prm{};
  double lin_dt = 0.0;
  void* blocks = nullptr;      // block-Jacobi factors (FP32), [number][n_el]
  void* blocks_raw = nullptr;  // unfactored blocks, [n_el][row][col]
  // face traces (field values at every face point) of the linearisation state
  void* trL = nullptr;
  // reduction scratch
  double* part = nullptr;
  size_t part_len = 0;
  double* red_out = nullptr;      // device [64]
  double* red_host = nullptr;     // pinned, device-mapped [80]
  double* red_dev_map = nullptr;  // device view of red_host
  // solver workspace
  void* gm = nullptr;             // whole-solve workspace (state and Krylov vectors)
  size_t gm_bytes = 0;
  void* eng = nullptr;            // whole-solve engine (one-instance batch), type-erased
  void (*eng_free)(void*) = nullptr;
};

namespace {

thread_local std::string g_err_no_ctx;

inline void hfree(void* p) {
  if (p) (void)hipFree(p);
}

int fail(bsw_ctx c, int code, const std::string& msg) {
  if (c) c->err = msg; else g_err_no_ctx = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t _e = (call);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail((ctx), BSW_E_HIP, std::string(#call) + ": " + hipGetErrorString(_e)); \
  } while (0)

template <class T>
int dev_alloc(bsw_ctx c, T** p, size_t count) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) return fail(c, BSW_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  return BSW_OK;
}

int combo_index(int dim, int P) {
  for (int k = 0; k < kNumCombos; ++k)
    if (kCombo[k][0] == dim && kCombo[k][1] == P) return k;
  return -1;
}

// ---------------------------------------------------------------- dispatch
template <class T, class F>
int dispatchT(int dim, int P, F& f) {
  if (dim == 1) {
    switch (P) {
      case 0: return f.template operator()<1, 0, T>();
      case 1: return f.template operator()<1, 1, T>();
      case 2: return f.template operator()<1, 2, T>();
      case 3: return f.template operator()<1, 3, T>();
      case 4: return f.template operator()<1, 4, T>();
    }
  } else {
    switch (P) {
      case 1: return f.template operator()<2, 1, T>();
      case 2: return f.template operator()<2, 2, T>();
      case 3: return f.template operator()<2, 3, T>();
    }
  }
  return BSW_E_ARG;
}

template <class F>
int dispatch(bsw_disc d, F&& f) {
  if (d->precision == BSW_FP64) return dispatchT<double>(d->mesh->dim, d->P, f);
  return dispatchT<float>(d->mesh->dim, d->P, f);
}

template <class T>
MeshView<T> view(bsw_disc d) {
  MeshView<T> v;
  v.n_el = (int)d->mesh->n_el;
  const DevMesh<T>* dm;
  if constexpr (sizeof(T) == 8) dm = &d->mesh->m64; else dm = &d->mesh->m32;
  v.dxi = dm->dxi; v.detJ = dm->detJ; v.nrm = dm->nrm; v.hlen = dm->hlen;
  v.nbr = d->mesh->nbr;
  v.vert = d->mesh->vert;
  v.bed = (const T*)d->bed;
  v.nmodes = d->nmode[0] | d->nmode[1] << 8 | d->nmode[2] << 16;
  return v;
}

template <class T>
DevParams<T> devparams(const bsw_params& p, double dt, const T* dirtab) {
  DevParams<T> q;
  q.g = (T)p.g;
  q.gc = (T)(p.g * std::cos(p.alpha));
  q.gs = (T)(p.g * std::sin(p.alpha));
  q.rho_inv = (T)(1.0 / p.rho);
  q.eta = (T)p.eta; q.s0 = (T)p.sigma0; q.gam = (T)p.gamma; q.bet = (T)p.beta;
  q.inv_dt = dt > 0 ? (T)(1.0 / dt) : T(0);
  q.reg = p.reg; q.bc = p.bc; q.jfrozen = p.jac_frozen != 0;
  q.dirtab = dirtab;
  return q;
}

// the Dirichlet states of p (tags 0..3) in the discretisation's device table,
// rewritten only when they change (after the stream has drained, so kernels
// already queued keep the values they were launched with)
void dirichlet_table(const bsw_params& p, double* v) {
  for (int k = 0; k < 7; ++k) v[k] = p.dirichlet[k];
  for (int t = 0; t < 3; ++t)
    for (int k = 0; k < 7; ++k) v[7 * (t + 1) + k] = p.dirichlet_tag[t][k];
}

template <class T>
int sync_dirtab(bsw_disc d, const bsw_params& p) {
  double v[28];
  dirichlet_table(p, v);
  if (d->dirtab_set && std::memcmp(v, d->dirtab_host, sizeof(v)) == 0) return BSW_OK;
  bsw_ctx c = d->mesh->ctx;
  T tv[28];
  for (int k = 0; k < 28; ++k) tv[k] = (T)v[k];
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(d->dirtab, tv, sizeof(tv), hipMemcpyHostToDevice));
  std::memcpy(d->dirtab_host, v, sizeof(v));
  d->dirtab_set = true;
  return BSW_OK;
}

int check_params(bsw_disc d, const bsw_params* p) {
  bsw_ctx c = d->mesh->ctx;
  if (!p) return fail(c, BSW_E_ARG, "params is null");
  if (p->reg < 1 || p->reg > 3) return fail(c, BSW_E_ARG, "reg must be 1, 2 or 3");
  if (p->bc < 1 || p->bc > 3) return fail(c, BSW_E_ARG, "bc must be 1 (wall), 2 (Neumann) or 3 (Dirichlet)");
  if (!(p->g > 0) || !(p->rho > 0) || p->eta < 0 || p->sigma0 < 0 || !(p->gamma > 0) || !(p->beta > 0))
    return fail(c, BSW_E_ARG, "need g, rho, gamma, beta > 0 and eta, sigma0 >= 0");
  if (p->reg != 3 && p->sigma0 > 0 && p->sigma0 < 0.5 / p->beta)
    return fail(c, BSW_E_ARG, "regularisations 1 and 2 need sigma0 >= 1/(2 beta)");
  return BSW_OK;
}

inline dim3 grid1(int64_t n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

// ---------------------------------------------------------------- reductions
constexpr int kRedThreads = 256;

__device__ __forceinline__ double red_op(double a, double b, int op) {
  return op == 0 ? a + b : (op == 1 ? fmax(a, b) : fmin(a, b));
}

// block-level reduction of NV values per thread into part[v * nblk + blockIdx.x]
template <int NV>
__device__ void block_reduce(double (&val)[NV], const int (&ops)[NV], double* part) {
  __shared__ double sh[NV][kRedThreads];
#pragma unroll
  for (int v = 0; v < NV; ++v) sh[v][threadIdx.x] = val[v];
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int v = 0; v < NV; ++v) sh[v][threadIdx.x] = red_op(sh[v][threadIdx.x], sh[v][threadIdx.x + s], ops[v]);
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int v = 0; v < NV; ++v) part[v * gridDim.x + blockIdx.x] = sh[v][0];
}

// final pass: out[v] = reduce(part[v][0..nblk)), one block per value, fixed order
__global__ void __launch_bounds__(kRedThreads) k_reduce_final(const double* __restrict__ part, int nblk,
                                                               const int* __restrict__ ops_unused, int op0,
                                                               int op1, int op2, int op3, double* out) {
  const int v = blockIdx.x;
  const int op = v == 0 ? op0 : (v == 1 ? op1 : (v == 2 ? op2 : op3));
  const double init = op == 0 ? 0.0 : (op == 1 ? -INFINITY : INFINITY);
  double acc = init;
  for (int i = threadIdx.x; i < nblk; i += kRedThreads) acc = red_op(acc, part[(size_t)v * nblk + i], op);
  __shared__ double sh[kRedThreads];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = red_op(sh[threadIdx.x], sh[threadIdx.x + s], op);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = sh[0];
}

// dot products of w with k vectors V[j] (stride ld) -> part[j][blk]; a grid
// row y == k (when present) gives w . w
template <class T>
__global__ void __launch_bounds__(kRedThreads) k_multidot(const T* __restrict__ V, size_t ld, const T* __restrict__ w,
                                                           int64_t n, int k, double* __restrict__ part) {
  const int j = blockIdx.y;
  const T* v = j < k ? V + (size_t)j * ld : w;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads)
    acc += (double)v[i] * (double)w[i];
  __shared__ double sh[kRedThreads];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)j * gridDim.x + blockIdx.x] = sh[0];
}

// W += alpha dW with max|alpha dW| and max|W| partials
template <class T>
__global__ void __launch_bounds__(kRedThreads) k_axpy_norms(T* __restrict__ W, const T* __restrict__ dW, double alpha,
                                                             int64_t n, double* part) {
  double v[2] = {0.0, 0.0};
  const int ops[2] = {1, 1};
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads) {
    const double d = alpha * (double)dW[i];
    const T wn = (T)((double)W[i] + d);
    W[i] = wn;
    v[0] = fmax(v[0], fabs(d));
    v[1] = fmax(v[1], fabs((double)wn));
  }
  block_reduce<2>(v, ops, part);
}

// mass, active area, max(|u| + sqrt(g h)), min h over volume points (Sec. 6)
template <int D, int P, class T>
__global__ void __launch_bounds__(kRedThreads) k_diag(const T* __restrict__ W, MeshView<T> m, double g, double thr,
                                                       double* part) {
  double v[4] = {0.0, 0.0, 0.0, INFINITY};
  const int ops[4] = {0, 0, 1, 2};
  for (int e = blockIdx.x * kRedThreads + threadIdx.x; e < m.n_el; e += gridDim.x * kRedThreads)
    diag_elem<D, P, T>(W, m, g, thr, e, v);
  block_reduce<4>(v, ops, part);
}

// L2 projection of an analytic initial condition (E = 0)
__device__ void ic_eval(const bsw_ic& ic, int dim, double x, double y, double& h, double& u, double& v) {
  u = 0.0; v = 0.0;
  const double pi = 3.14159265358979323846;
  switch (ic.kind) {
    case BSW_IC_CONST: h = ic.a; u = ic.b; v = ic.c; break;
    case BSW_IC_STEP_X: h = x < ic.x0 ? ic.a : ic.b; break;
    case BSW_IC_MOUND: {
      const double r2 = (x - ic.x0) * (x - ic.x0) + (dim == 2 ? (y - ic.y0) * (y - ic.y0) : 0.0);
      h = ic.a + ic.b * exp(-r2 / ic.d);
    } break;
    case BSW_IC_DISK: {
      const double r2 = (x - ic.x0) * (x - ic.x0) + (dim == 2 ? (y - ic.y0) * (y - ic.y0) : 0.0);
      h = r2 < ic.r * ic.r ? ic.a : ic.b;
    } break;
    case BSW_IC_SINE_U: h = ic.a; u = ic.b * sin(pi * x / ic.L); break;
    case BSW_IC_LINEAR_X: h = ic.a + ic.b * x; break;
    case BSW_IC_SURFACE: h = ic.a + ic.b * x; break;  // the bed is subtracted after the projection
    case BSW_IC_SHEAR_Y: h = ic.a; u = ic.b * cos(pi * y / ic.L); break;
    case BSW_IC_VORTEX:
      h = ic.a;
      u = ic.b * sin(pi * x / ic.L) * cos(pi * y / ic.L);
      v = -ic.b * cos(pi * x / ic.L) * sin(pi * y / ic.L);
      break;
    default: h = 1.0;
  }
}

template <int D, int P, class T>
__global__ void __launch_bounds__(256) k_project_ic(T* __restrict__ W, MeshView<T> m, bsw_ic ic,
                                                     const double* __restrict__ qxi) {
  using S = Shape<D, P>;
  const Tab<D, P, T>& tb = tab<D, P, T>();
  const int n = m.n_el;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double acc[1 + D][S::NP];
#pragma unroll
  for (int f = 0; f <= D; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) acc[f][i] = 0.0;
  double vx[D + 1][D];
#pragma unroll
  for (int k = 0; k <= D; ++k)
#pragma unroll
    for (int a = 0; a < D; ++a) vx[k][a] = m.vert[(size_t)(k * D + a) * n + e];
#pragma unroll
  for (int q = 0; q < S::NQ; ++q) {
    double x, y = 0.0;
    if (D == 1) {
      x = vx[0][0] + 0.5 * (qxi[2 * q] + 1.0) * (vx[1][0] - vx[0][0]);
    } else {
      const double s = qxi[2 * q], t = qxi[2 * q + 1];
      x = vx[0][0] + s * (vx[1][0] - vx[0][0]) + t * (vx[D][0] - vx[0][0]);
      y = vx[0][D - 1] + s * (vx[1][D - 1] - vx[0][D - 1]) + t * (vx[D][D - 1] - vx[0][D - 1]);
    }
    double h, u, v;
    ic_eval(ic, D, x, y, h, u, v);
    const double val[3] = {h, u, v};
#pragma unroll
    for (int i = 0; i < S::NP; ++i) {
      const double c = (double)tb.qw[q] * (double)tb.phi[q][i];
#pragma unroll
      for (int f = 0; f <= D; ++f) acc[f][i] += c * val[f];
    }
  }
  if (ic.kind == BSW_IC_SURFACE && m.bed) {
    // h = surface - H mode by mode: as continuous as the bed
#pragma unroll
    for (int i = 0; i < S::NP; ++i) acc[0][i] -= (double)m.bed[(size_t)i * n + e];
  }
  // fields of lower order keep their first N(m) modes: the L2 projection onto
  // their space (orthonormal, degree-ordered basis)
#pragma unroll
  for (int f = 0; f <= D; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i)
      if (row_unused<D, T>(m, f, i)) acc[f][i] = 0.0;
  if (ic.kind != BSW_IC_SURFACE) {
    // positivity of the projected depth: where it drops below a tenth of the
    // element mean at a volume or face point, scale the higher depth modes so
    // the minimum is a tenth of the mean (mean and mass unchanged)
    const double mean = acc[0][0] * (double)tb.phi[0][0];
    double mn = INFINITY;
    for (int q = 0; q < S::NQ; ++q) {
      double s = 0.0;
      for (int i = 0; i < S::NP; ++i) s += (double)tb.phi[q][i] * acc[0][i];
      mn = fmin(mn, s);
    }
    for (int fc = 0; fc < S::NFC; ++fc)
      for (int r = 0; r < S::NFQ; ++r) {
        double s = 0.0;
        for (int i = 0; i < S::NP; ++i) s += (double)tb.fphi[fc][r][i] * acc[0][i];
        mn = fmin(mn, s);
      }
    if (mean > 0.0 && mn < 0.1 * mean) {
      const double theta = 0.9 * mean / (mean - mn);
      for (int i = 1; i < S::NP; ++i) acc[0][i] *= theta;
    }
  }
#pragma unroll
  for (int f = 0; f < S::NF; ++f)
#pragma unroll
    for (int i = 0; i < S::NP; ++i) W[(size_t)(f * S::NP + i) * n + e] = f <= D ? (T)acc[f][i] : T(0);
}

// Bed interpolant (Eq. Sterm, Sec. 5): H at the NN order-m0 nodes of element e
// (reference coordinates xi[2k], xi[2k+1], FP64), then the modal coefficients
// c = Vinv H(nodes) of the first NN modes; the higher modes are zero.
__device__ double bed_eval(const bsw_bed& b, int dim, double x, double y) {
  switch (b.kind) {
    case BSW_BED_COS: return b.a * cos(b.kx * x) * (dim == 2 ? cos(b.ky * y) : 1.0);
    case BSW_BED_GAUSS: {
      const double r2 = (x - b.x0) * (x - b.x0) + (dim == 2 ? (y - b.y0) * (y - b.y0) : 0.0);
      return b.a * exp(-r2 / b.d);
    }
    default: return 0.0;
  }
}

template <int D, int P, class T>
__global__ void __launch_bounds__(256) k_bed_interp(T* __restrict__ H, MeshView<T> m, bsw_bed bed, int nn,
                                                     const double* __restrict__ tab) {
  using S = Shape<D, P>;
  const int n = m.n_el;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double* xi = tab;             // [nn][2]
  const double* vinv = tab + 2 * nn;  // [nn][nn], row = mode
  double vx[D + 1][D];
#pragma unroll
  for (int k = 0; k <= D; ++k)
#pragma unroll
    for (int a = 0; a < D; ++a) vx[k][a] = m.vert[(size_t)(k * D + a) * n + e];
  double hv[S::NP];
#pragma unroll
  for (int j = 0; j < S::NP; ++j) {
    hv[j] = 0.0;
    if (j < nn) {
      double x, y = 0.0;
      if (D == 1) {
        x = vx[0][0] + 0.5 * (xi[2 * j] + 1.0) * (vx[1][0] - vx[0][0]);
      } else {
        const double s = xi[2 * j], t = xi[2 * j + 1];
        x = vx[0][0] + s * (vx[1][0] - vx[0][0]) + t * (vx[D][0] - vx[0][0]);
        y = vx[0][D - 1] + s * (vx[1][D - 1] - vx[0][D - 1]) + t * (vx[D][D - 1] - vx[0][D - 1]);
      }
      hv[j] = bed_eval(bed, D, x, y);
    }
  }
#pragma unroll
  for (int i = 0; i < S::NP; ++i) {
    double c = 0.0;
    if (i < nn)
      for (int j = 0; j < nn; ++j) c += vinv[i * nn + j] * hv[j];
    H[(size_t)i * n + e] = (T)c;
  }
}

// ---------------------------------------------------------------- reductions (host helpers)
int ensure_part(bsw_disc d, size_t len) {
  if (d->part_len >= len) return BSW_OK;
  bsw_ctx c = d->mesh->ctx;
  hfree(d->part);
  d->part = nullptr;
  d->part_len = 0;
  if (int rc = dev_alloc(c, &d->part, len)) return rc;
  d->part_len = len;
  return BSW_OK;
}

int red_blocks(int64_t n) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + kRedThreads - 1) / kRedThreads)); }

// finish a partial reduction of nv values (partials part[v * nblk + b]) into
// the device values dev_out[0..nv) and host out[]
int finish_into(bsw_disc d, const double* part, double* dev_out, int nblk, int nv, const int* ops,
                double* host_out) {
  bsw_ctx c = d->mesh->ctx;
  hipLaunchKernelGGL(k_reduce_final, dim3(nv), dim3(kRedThreads), 0, c->stream, part, nblk, nullptr, ops[0],
                     nv > 1 ? ops[1] : 0, nv > 2 ? ops[2] : 0, nv > 3 ? ops[3] : 0, dev_out);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(d->red_host, dev_out, sizeof(double) * nv, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < nv; ++k) host_out[k] = d->red_host[k];
  return BSW_OK;
}

int finish(bsw_disc d, int nblk, int nv, const int* ops, double* host_out) {
  return finish_into(d, d->part, d->red_out, nblk, nv, ops, host_out);
}

// --------------------------------------------------------------- kernel launchers
// the element-pass variant the single-call entry points launch: the one
// bsw_tile_policy forces, else variant 1 (defined with the autotuner)
int single_call_variant();

struct OpLaunch {
  bsw_disc d; const bsw_params* p; double dt; const void* W; const void* bold; void* R;
  template <int D, int P, class T, int V>
  void launch(hipStream_t st, const MeshView<T>& m, const DevParams<T>& prm) {
    hipLaunchKernelGGL((k_elem<D, P, T, 0, V>), grid1(m.n_el, etile_eb<D, P, V>()), dim3(etile_nt<D, V>()), 0, st,
                       (const T*)W, (const T*)nullptr, (const T*)bold, (T*)R, (const T*)nullptr, m, prm);
  }
  template <int D, int P, class T>
  int operator()() {
    auto m = view<T>(d);
    hipStream_t st = d->mesh->ctx->stream;
    if (int rc = sync_dirtab<T>(d, *p)) return rc;
    // one element pass: it evaluates the neighbours' side of W itself
    const auto prm = devparams<T>(*p, dt, (const T*)d->dirtab);
    switch (single_call_variant()) {
      case 0: launch<D, P, T, 0>(st, m, prm); break;
      case 2: launch<D, P, T, 2>(st, m, prm); break;
      default: launch<D, P, T, 1>(st, m, prm);
    }
    HIPCHK(d->mesh->ctx, hipGetLastError());
    return BSW_OK;
  }
};

struct StepBeginLaunch {
  bsw_disc d; const bsw_params* p; double dt; const void* W; void* bold;
  template <int D, int P, class T>
  int operator()() {
    auto m = view<T>(d);
    hipLaunchKernelGGL((k_step_begin<D, P, T>), grid1(m.n_el), dim3(256), 0, d->mesh->ctx->stream, (const T*)W,
                       (T*)bold, m, devparams<T>(*p, dt, (const T*)nullptr));
    HIPCHK(d->mesh->ctx, hipGetLastError());
    return BSW_OK;
  }
};

struct JacApplyLaunch {
  bsw_disc d; const void* x; void* y;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;  // optional: timestamps of this dispatch
  // one element pass (it evaluates the neighbours' side of x itself); with
  // events, ev_start and ev_stop stamp its start and end
  template <int D, int P, class T, int V>
  void launch(hipStream_t st, const MeshView<T>& m, const DevParams<T>& prm) {
    hipExtLaunchKernelGGL((k_elem<D, P, T, 1, V>), grid1(m.n_el, etile_eb<D, P, V>()), dim3(etile_nt<D, V>()), 0, st,
                          ev_start, ev_stop, 0, (const T*)d->lin_W, (const T*)x, (const T*)nullptr, (T*)y,
                          (const T*)d->trL, m, prm);
  }
  template <int D, int P, class T>
  int operator()() {
    auto m = view<T>(d);
    hipStream_t st = d->mesh->ctx->stream;
    if (int rc = sync_dirtab<T>(d, d->lin_prm)) return rc;
    const auto prm = devparams<T>(d->lin_prm, d->lin_dt, (const T*)d->dirtab);
    switch (single_call_variant()) {
      case 0: launch<D, P, T, 0>(st, m, prm); break;
      case 2: launch<D, P, T, 2>(st, m, prm); break;
      default: launch<D, P, T, 1>(st, m, prm);
    }
    HIPCHK(d->mesh->ctx, hipGetLastError());
    return BSW_OK;
  }
};

struct LinearizeLaunch {
  bsw_disc d;
  template <int D, int P, class T>
  int operator()() {
    using S = Shape<D, P>;
    auto m = view<T>(d);
    bsw_ctx c = d->mesh->ctx;
    if (int rc = sync_dirtab<T>(d, d->lin_prm)) return rc;
    hipLaunchKernelGGL((k_trace<D, P, T>), grid1((int64_t)S::NF * S::NFC * m.n_el), dim3(256), 0, c->stream,
                       (const T*)d->lin_W, (T*)d->trL, m.n_el);
    const auto prm = devparams<T>(d->lin_prm, d->lin_dt, (const T*)d->dirtab);
    // triangles: only the parts the factors read (bsw_jacobian_blocks
    // assembles whole blocks when asked)
    if constexpr (D == 2)
      hipLaunchKernelGGL((k_jac_blocks_tri<P, T, false>), dim3(m.n_el), dim3(JB2<P>::NT), 0, c->stream,
                         (const T*)d->lin_W, (const T*)d->trL, (T*)d->blocks_raw, m, prm);
    else
      hipLaunchKernelGGL((k_jac_columns<D, P, T>), dim3(cols_tiles_for(S::BS, m.n_el)), dim3(256), 0, c->stream,
                         (const T*)d->lin_W, (const T*)d->trL, (T*)d->blocks_raw, m, prm);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL((k_schur_build<D, P, T>), dim3((unsigned)((m.n_el + kSchurEPB - 1) / kSchurEPB)), dim3(256), 0,
                       c->stream, (const T*)d->blocks_raw, (float*)d->blocks, m.n_el);
    HIPCHK(c, hipGetLastError());
    return BSW_OK;
  }
};

// whole diagonal blocks of triangles from the linearisation state (the
// linearisation itself assembles only the parts its factors read)
struct BlocksLaunch {
  bsw_disc d;
  template <int D, int P, class T>
  int operator()() {
    if constexpr (D == 2) {
      using S = Shape<D, P>;
      auto m = view<T>(d);
      bsw_ctx c = d->mesh->ctx;
      if (int rc = sync_dirtab<T>(d, d->lin_prm)) return rc;
      hipLaunchKernelGGL((k_trace<D, P, T>), grid1((int64_t)S::NF * S::NFC * m.n_el), dim3(256), 0, c->stream,
                         (const T*)d->lin_W, (T*)d->trL, m.n_el);
      const auto prm = devparams<T>(d->lin_prm, d->lin_dt, (const T*)d->dirtab);
      hipLaunchKernelGGL((k_jac_blocks_tri<P, T, true>), dim3(m.n_el), dim3(JB2<P>::NT), 0, c->stream,
                         (const T*)d->lin_W, (const T*)d->trL, (T*)d->blocks_raw, m, prm);
      HIPCHK(c, hipGetLastError());
    }
    return BSW_OK;
  }
};

struct PrecLaunch {
  bsw_disc d; const void* x; void* y;
  template <int D, int P, class T>
  int operator()() {
    auto m = view<T>(d);
    hipLaunchKernelGGL((k_schur_apply<D, P, T>), dim3((unsigned)((m.n_el + kPrecEB - 1) / kPrecEB)), dim3(256), 0,
                       d->mesh->ctx->stream, (const float*)d->blocks, (const T*)x, (T*)y, m, d->lin_prm.bc);
    HIPCHK(d->mesh->ctx, hipGetLastError());
    return BSW_OK;
  }
};

struct DiagLaunch {
  bsw_disc d; const bsw_params* p; const void* W; int nblk; double* part;
  template <int D, int P, class T>
  int operator()() {
    auto m = view<T>(d);
    const double thr = p->sigma0 / p->gamma;
    hipLaunchKernelGGL((k_diag<D, P, T>), dim3(nblk), dim3(kRedThreads), 0, d->mesh->ctx->stream, (const T*)W, m,
                       p->g, thr, part);
    HIPCHK(d->mesh->ctx, hipGetLastError());
    return BSW_OK;
  }
};

struct ICLaunch {
  bsw_disc d; bsw_ic ic; void* W; double* qxi;
  template <int D, int P, class T>
  int operator()() {
    auto m = view<T>(d);
    hipLaunchKernelGGL((k_project_ic<D, P, T>), grid1(m.n_el), dim3(256), 0, d->mesh->ctx->stream, (T*)W, m, ic, qxi);
    HIPCHK(d->mesh->ctx, hipGetLastError());
    return BSW_OK;
  }
};

struct BedLaunch {
  bsw_disc d; bsw_bed bed; void* H; int nn; double* tab;
  template <int D, int P, class T>
  int operator()() {
    auto m = view<T>(d);
    hipLaunchKernelGGL((k_bed_interp<D, P, T>), grid1(m.n_el), dim3(256), 0, d->mesh->ctx->stream, (T*)H, m, bed, nn,
                       tab);
    HIPCHK(d->mesh->ctx, hipGetLastError());
    return BSW_OK;
  }
};

// Order-m interpolation nodes shared by neighbouring elements, as reference
// coordinates: Gauss-Lobatto points on [-1, 1]; on the unit triangle the
// vertices, each edge's interior Gauss-Lobatto points (symmetric about the
// edge midpoint, so both elements of an edge meet the same physical points)
// and the centroid at m = 3.
bool bed_nodes(int dim, int m, std::vector<double>& xi) {
  std::vector<double> t;  // interior Lobatto points: the roots of P_m'
  if (m == 2) t = {0.0};
  else if (m == 3) t = {-std::sqrt(0.2), std::sqrt(0.2)};
  else if (m == 4) t = {-std::sqrt(3.0 / 7.0), 0.0, std::sqrt(3.0 / 7.0)};
  else if (m != 1) return false;
  xi.clear();
  if (dim == 1) {
    xi.insert(xi.end(), {-1.0, 0.0});
    for (double v : t) xi.insert(xi.end(), {v, 0.0});
    xi.insert(xi.end(), {1.0, 0.0});
    return true;
  }
  if (m > 3) return false;
  const double V[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
  for (auto& v : V) xi.insert(xi.end(), {v[0], v[1]});
  for (int f = 0; f < 3; ++f)
    for (double v : t) {
      const double s = 0.5 * (v + 1.0);
      const double* A = V[f];
      const double* B = V[(f + 1) % 3];
      xi.insert(xi.end(), {A[0] + s * (B[0] - A[0]), A[1] + s * (B[1] - A[1])});
    }
  if (m == 3) xi.insert(xi.end(), {1.0 / 3.0, 1.0 / 3.0});
  return true;
}

// In-place inverse of a small dense matrix (Gauss-Jordan, partial pivoting).
bool invert_small(int n, std::vector<double>& A) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int pv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[pv * n + k])) pv = i;
    if (A[pv * n + k] == 0.0) return false;
    for (int j = 0; j < n; ++j) { std::swap(A[k * n + j], A[pv * n + j]); std::swap(I[k * n + j], I[pv * n + j]); }
    const double inv = 1.0 / A[k * n + k];
    for (int j = 0; j < n; ++j) { A[k * n + j] *= inv; I[k * n + j] *= inv; }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = A[i * n + k];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) { A[i * n + j] -= f * A[k * n + j]; I[i * n + j] -= f * I[k * n + j]; }
    }
  }
  A.swap(I);
  return true;
}

// ---------------------------------------------------------------- table staging
template <int D, int P, class T>
void fill_tab(const RefElement& R, Tab<D, P, T>& t) {
  using S = Shape<D, P>;
  for (int q = 0; q < S::NQ; ++q) {
    t.qw[q] = (T)R.qw[q];
    for (int i = 0; i < S::NP; ++i) {
      t.phi[q][i] = (T)R.phi[q * S::NP + i];
      for (int r = 0; r < D; ++r) t.dphi[q][i][r] = (T)R.dphi[(q * S::NP + i) * 2 + r];
    }
  }
  for (int f = 0; f < S::NFC; ++f)
    for (int r = 0; r < S::NFQ; ++r)
      for (int i = 0; i < S::NP; ++i) t.fphi[f][r][i] = (T)R.fphi[(f * S::NFQ + r) * S::NP + i];
  for (int r = 0; r < S::NFQ; ++r) t.fw[r] = (T)R.fw[r];
}

struct StageTables {
  bsw_disc d;
  template <int D, int P, class T>
  int operator()() {
    bsw_ctx c = d->mesh->ctx;
    const RefElement& R = d->ref;
    if (R.np != Shape<D, P>::NP || R.nq != Shape<D, P>::NQ || R.nfq != Shape<D, P>::NFQ)
      return fail(c, BSW_E_ARG, "reference element does not match the compiled shape");
    Tab<D, P, T> t;
    fill_tab<D, P, T>(R, t);
    HIPCHK(c, hipMemcpyToSymbol(HIP_SYMBOL(c_tables), &t, sizeof(t), tab_offset_rt(D, P, sizeof(T) == 4),
                                hipMemcpyHostToDevice));
    return BSW_OK;
  }
};

}  // namespace

// ====================================================================== C ABI
extern "C" {

int bsw_ctx_create(int device, void* hip_stream, bsw_ctx* out) {
  if (!out) return fail(nullptr, BSW_E_ARG, "out is null");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(nullptr, BSW_E_ARG, "no such HIP device");
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, BSW_E_HIP, "hipSetDevice failed");
  bsw_ctx c = new bsw_ctx_s();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  // this device's copy of the scratch array, looked up once per device with
  // the device current (the array's name is a host-side stand-in; kernels and
  // copies must use this address)
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device >= kMaxScratchDevices) {
      delete c;
      return fail(nullptr, BSW_E_ARG, "device index beyond the scratch table");
    }
    if (!g_scratch_dev[device]) {
      void* sp = nullptr;
      const hipError_t se = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
      if (se != hipSuccess || !sp) {
        delete c;
        return fail(nullptr, BSW_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(se));
      }
      g_scratch_dev[device] = (double*)sp;
    }
    c->scratch = g_scratch_dev[device];
  }
  *out = c;
  return BSW_OK;
}

int bsw_ctx_destroy(bsw_ctx c) {
  delete c;
  return BSW_OK;
}

const char* bsw_last_error(bsw_ctx c) { return c ? c->err.c_str() : g_err_no_ctx.c_str(); }

int bsw_mesh_upload(bsw_ctx c, int dim, int64_t n_vert, const double* xy, int64_t n_el, const int32_t* e2v,
                    bsw_mesh* out) {
  if (!c || !out || !xy || !e2v) return fail(c, BSW_E_ARG, "null argument");
  if ((dim != 1 && dim != 2) || n_vert < 2 || n_el < 1 || n_el > (int64_t(1) << 29))
    return fail(c, BSW_E_ARG, "bad mesh sizes");
  HIPCHK(c, hipSetDevice(c->device));
  const int nvpe = dim + 1, nfc = dim + 1;
  for (int64_t k = 0; k < n_el * nvpe; ++k)
    if (e2v[k] < 0 || e2v[k] >= n_vert) return fail(c, BSW_E_ARG, "vertex index out of range");
  const int64_t n = n_el;
  std::vector<double> dxi(dim * dim * n), detJ(n), nrm(nfc * dim * n), hlen(nfc * n), vert((dim + 1) * dim * n);
  std::vector<int> nbr(nfc * n, -1);
  double hmin = 1e300, meas = 0.0;
  for (int64_t e = 0; e < n; ++e) {
    const int32_t* v = e2v + e * nvpe;
    for (int k = 0; k <= dim; ++k)
      for (int a = 0; a < dim; ++a) vert[(k * dim + a) * n + e] = xy[(int64_t)v[k] * dim + a];
    if (dim == 1) {
      const double L = xy[v[1]] - xy[v[0]];
      if (!(L > 0)) return fail(c, BSW_E_MESH, "non-positive segment length");
      detJ[e] = 0.5 * L;
      dxi[e] = 2.0 / L;
      nrm[0 * n + e] = -1.0;
      nrm[1 * n + e] = 1.0;
      hlen[0 * n + e] = hlen[1 * n + e] = 1.0;
      hmin = std::min(hmin, L);
      meas += L;
    } else {
      const double x0 = xy[2 * v[0]], y0 = xy[2 * v[0] + 1];
      const double x1 = xy[2 * v[1]], y1 = xy[2 * v[1] + 1];
      const double x2 = xy[2 * v[2]], y2 = xy[2 * v[2] + 1];
      const double j11 = x1 - x0, j12 = x2 - x0, j21 = y1 - y0, j22 = y2 - y0;
      const double det = j11 * j22 - j12 * j21;
      if (!(det > 0)) return fail(c, BSW_E_MESH, "triangle with non-positive orientation");
      detJ[e] = det;
      // inverse of the affine map's Jacobian: rows (dxi/dx, dxi/dy), (deta/dx, deta/dy)
      dxi[0 * n + e] = j22 / det;
      dxi[1 * n + e] = -j12 / det;
      dxi[2 * n + e] = -j21 / det;
      dxi[3 * n + e] = j11 / det;
      const double X[3] = {x0, x1, x2}, Y[3] = {y0, y1, y2};
      double lmax = 0.0;
      for (int f = 0; f < 3; ++f) {
        const double ex = X[(f + 1) % 3] - X[f], ey = Y[(f + 1) % 3] - Y[f];
        const double L = std::sqrt(ex * ex + ey * ey);
        nrm[(f * 2 + 0) * n + e] = ey / L;
        nrm[(f * 2 + 1) * n + e] = -ex / L;
        hlen[f * n + e] = 0.5 * L;
        lmax = std::max(lmax, L);
      }
      hmin = std::min(hmin, det / lmax);
      meas += 0.5 * det;
    }
  }
  // faces: key = sorted vertex pair (2-D) or the vertex (1-D)
  std::unordered_map<uint64_t, int64_t> open;
  open.reserve((size_t)(n * nfc));
  for (int64_t e = 0; e < n; ++e)
    for (int f = 0; f < nfc; ++f) {
      const int32_t* v = e2v + e * nvpe;
      uint64_t key;
      if (dim == 1) key = (uint64_t)v[f];
      else {
        const uint64_t a = (uint64_t)v[f], b = (uint64_t)v[(f + 1) % 3];
        key = std::min(a, b) * (uint64_t)n_vert + std::max(a, b);
      }
      auto it = open.find(key);
      if (it == open.end()) {
        open.emplace(key, e * nfc + f);
      } else {
        const int64_t other = it->second;
        if (other < 0) return fail(c, BSW_E_MESH, "face shared by more than two elements");
        const int64_t oe = other / nfc;
        const int of = (int)(other % nfc);
        nbr[f * n + e] = (int)(oe * 4 + of);
        nbr[of * n + oe] = (int)(e * 4 + f);
        it->second = -1;
      }
    }
  bsw_mesh M = new bsw_mesh_s();
  M->ctx = c; M->dim = dim; M->nfc = nfc; M->n_el = n; M->n_vert = n_vert; M->hmin = hmin; M->measure = meas;
  auto up = [&](auto** dst, auto& src) -> int {
    using V = std::remove_pointer_t<std::remove_reference_t<decltype(*dst)>>;
    if (int rc = dev_alloc(c, dst, src.size())) return rc;
    HIPCHK(c, hipMemcpy(*dst, src.data(), sizeof(V) * src.size(), hipMemcpyHostToDevice));
    return BSW_OK;
  };
  int rc = BSW_OK;
  if (!rc) rc = up(&M->nbr, nbr);
  if (!rc) rc = up(&M->vert, vert);
  if (!rc) rc = up(&M->m64.dxi, dxi);
  if (!rc) rc = up(&M->m64.detJ, detJ);
  if (!rc) rc = up(&M->m64.nrm, nrm);
  if (!rc) rc = up(&M->m64.hlen, hlen);
  if (rc) { bsw_mesh_destroy(M); return rc; }
  M->h_dxi = std::move(dxi); M->h_detJ = std::move(detJ); M->h_nrm = std::move(nrm); M->h_hlen = std::move(hlen);
  M->h_nbr = std::move(nbr);
  *out = M;
  return BSW_OK;
}

int bsw_mesh_set_boundary(bsw_mesh M, const int8_t* face_bc) {
  if (!M) return fail(nullptr, BSW_E_ARG, "null mesh");
  bsw_ctx c = M->ctx;
  const int64_t n = M->n_el;
  const int nfc = M->nfc;
  std::vector<int> nbr(M->h_nbr);
  for (int64_t e = 0; e < n; ++e)
    for (int f = 0; f < nfc; ++f) {
      const int code = face_bc ? (int)face_bc[e * nfc + f] : 0;
      if (code < 0 || code > 15) return fail(c, BSW_E_ARG, "boundary codes must be in 0..15");
      int& v = nbr[(size_t)f * n + e];
      if (v < 0) v = -1 - code;
    }
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipMemcpy(M->nbr, nbr.data(), sizeof(int) * nbr.size(), hipMemcpyHostToDevice));
  return BSW_OK;
}

int bsw_mesh_destroy(bsw_mesh M) {
  if (!M) return BSW_OK;
  hfree(M->nbr); hfree(M->vert);
  hfree(M->m64.dxi); hfree(M->m64.detJ); hfree(M->m64.nrm); hfree(M->m64.hlen);
  hfree(M->m32.dxi); hfree(M->m32.detJ); hfree(M->m32.nrm); hfree(M->m32.hlen);
  delete M;
  return BSW_OK;
}

int bsw_disc_create(bsw_mesh M, int P, int precision, bsw_disc* out) {
  if (!M || !out) return fail(M ? M->ctx : nullptr, BSW_E_ARG, "null argument");
  bsw_ctx c = M->ctx;
  if (precision != BSW_FP64 && precision != BSW_FP32) return fail(c, BSW_E_ARG, "precision must be FP64 or FP32");
  if (combo_index(M->dim, P) < 0) return fail(c, BSW_E_ARG, "unsupported order for this dimension");
  HIPCHK(c, hipSetDevice(c->device));
  bsw_disc d = new bsw_disc_s();
  d->mesh = M; d->P = P; d->precision = precision;
  d->wsize = precision == BSW_FP64 ? 8 : 4;
  if (!build_reference(M->dim, P, d->ref)) { delete d; return fail(c, BSW_E_ARG, "reference element"); }
  d->bs = d->ref.nf * d->ref.np;
  d->nmode[0] = d->nmode[1] = d->nmode[2] = d->ref.np;
  // FP32 geometry view on first use
  if (precision == BSW_FP32 && !M->m32.dxi) {
    auto upf = [&](float** dst, const std::vector<double>& src) -> int {
      std::vector<float> tmp(src.begin(), src.end());
      if (int rc = dev_alloc(c, dst, tmp.size())) return rc;
      HIPCHK(c, hipMemcpy(*dst, tmp.data(), sizeof(float) * tmp.size(), hipMemcpyHostToDevice));
      return BSW_OK;
    };
    int rc = upf(&M->m32.dxi, M->h_dxi);
    if (!rc) rc = upf(&M->m32.detJ, M->h_detJ);
    if (!rc) rc = upf(&M->m32.nrm, M->h_nrm);
    if (!rc) rc = upf(&M->m32.hlen, M->h_hlen);
    if (rc) { delete d; return rc; }
  }
  const int ci = combo_index(M->dim, P);
  if (!c->tables_staged[precision][ci]) {
    StageTables st{d};
    if (int rc = dispatch(d, st)) { delete d; return rc; }
    c->tables_staged[precision][ci] = true;
  }
  const size_t ntr = (size_t)d->ref.nf * d->ref.nfc * d->ref.nfq * M->n_el * d->wsize;
  int rc = BSW_OK;
  if (hipMalloc(&d->trL, ntr) != hipSuccess) rc = fail(c, BSW_E_OOM, "face-trace storage");
  if (!rc) rc = dev_alloc(c, &d->red_out, 64);
  if (!rc && hipMalloc(&d->dirtab, 28 * d->wsize) != hipSuccess) rc = fail(c, BSW_E_OOM, "Dirichlet table");
  if (!rc && hipHostMalloc((void**)&d->red_host, 80 * sizeof(double), hipHostMallocMapped) != hipSuccess)
    rc = fail(c, BSW_E_OOM, "hipHostMalloc");
  if (!rc && hipHostGetDevicePointer((void**)&d->red_dev_map, d->red_host, 0) != hipSuccess)
    rc = fail(c, BSW_E_HIP, "hipHostGetDevicePointer");
  if (rc) { bsw_disc_destroy(d); return rc; }
  *out = d;
  return BSW_OK;
}

int bsw_disc_destroy(bsw_disc d) {
  if (!d) return BSW_OK;
  hfree(d->blocks); hfree(d->blocks_raw); hfree(d->part); hfree(d->red_out);
  hfree(d->trL);
  if (d->eng) d->eng_free(d->eng);
  hfree(d->gm); hfree(d->dirtab);
  if (d->red_host) (void)hipHostFree(d->red_host);
  delete d;
  return BSW_OK;
}

int bsw_disc_info(bsw_disc d, int64_t* info) {
  if (!d || !info) return BSW_E_ARG;
  info[0] = d->mesh->dim; info[1] = d->P; info[2] = d->ref.np; info[3] = d->ref.nq; info[4] = d->ref.nfq;
  info[5] = d->ref.nfc; info[6] = d->ref.nf; info[7] = d->mesh->n_el;
  return BSW_OK;
}

int64_t bsw_state_len(bsw_disc d) { return d ? (int64_t)d->bs * d->mesh->n_el : -1; }

int bsw_project_ic(bsw_disc d, const bsw_ic* ic, void* W) {
  if (!d || !ic || !W) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "null argument");
  bsw_ctx c = d->mesh->ctx;
  double* qxi = nullptr;
  if (int rc = dev_alloc(c, &qxi, d->ref.qxi.size())) return rc;
  HIPCHK(c, hipMemcpy(qxi, d->ref.qxi.data(), sizeof(double) * d->ref.qxi.size(), hipMemcpyHostToDevice));
  ICLaunch L{d, *ic, W, qxi};
  int rc = dispatch(d, L);
  (void)hipStreamSynchronize(c->stream);
  hfree(qxi);
  return rc;
}

int bsw_bed_interpolate(bsw_disc d, const bsw_bed* bed, void* H) {
  if (!d || !bed || !H) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "null argument");
  bsw_ctx c = d->mesh->ctx;
  const int dim = d->mesh->dim;
  const int m = bed->order > 0 ? bed->order : d->P;
  if (m < 1 || m > d->P) return fail(c, BSW_E_ARG, "bed order must be in 1..P");
  if (bed->kind < BSW_BED_FLAT || bed->kind > BSW_BED_GAUSS) return fail(c, BSW_E_ARG, "unknown bed kind");
  if (bed->kind == BSW_BED_GAUSS && !(bed->d > 0)) return fail(c, BSW_E_ARG, "GAUSS bed needs d > 0");
  std::vector<double> xi;
  if (!bed_nodes(dim, m, xi)) return fail(c, BSW_E_ARG, "bed order not supported for this element");
  const int nn = (int)xi.size() / 2;
  const int nm = dim == 1 ? m + 1 : (m + 1) * (m + 2) / 2;
  if (nn != nm || nm > d->ref.np) return fail(c, BSW_E_ARG, "bed node count");
  // Vandermonde of the first nm modes (they span the degree-m polynomials:
  // both bases are ordered by total degree) at the nodes, inverted
  std::vector<double> V((size_t)nn * nn), phi(d->ref.np);
  for (int j = 0; j < nn; ++j) {
    eval_basis(dim, d->P, xi[2 * j], xi[2 * j + 1], phi.data(), nullptr);
    for (int k = 0; k < nn; ++k) V[(size_t)j * nn + k] = phi[k];
  }
  if (!invert_small(nn, V)) return fail(c, BSW_E_ARG, "singular bed interpolation nodes");
  std::vector<double> host(xi);
  host.insert(host.end(), V.begin(), V.end());
  double* tab = nullptr;
  if (int rc = dev_alloc(c, &tab, host.size())) return rc;
  hipError_t he = hipMemcpyAsync(tab, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice, c->stream);
  int rc = BSW_OK;
  if (he != hipSuccess) {
    rc = fail(c, BSW_E_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(he));
  } else {
    BedLaunch L{d, *bed, H, nn, tab};
    rc = dispatch(d, L);
  }
  (void)hipStreamSynchronize(c->stream);
  hfree(tab);
  return rc;
}

int bsw_disc_set_orders(bsw_disc d, int m1, int m2, int m3) {
  if (!d) return fail(nullptr, BSW_E_ARG, "null discretisation");
  const int m[3] = {m1, m2, m3};
  for (int k = 0; k < 3; ++k)
    if (m[k] < 0 || m[k] > d->P) return fail(d->mesh->ctx, BSW_E_ARG, "orders must be in 0..P");
  for (int k = 0; k < 3; ++k) d->nmode[k] = d->mesh->dim == 1 ? m[k] + 1 : (m[k] + 1) * (m[k] + 2) / 2;
  d->lin_W = nullptr;  // the Jacobian's trivial rows moved
  return BSW_OK;
}

int bsw_disc_set_bed(bsw_disc d, const void* H) {
  if (!d) return fail(nullptr, BSW_E_ARG, "null discretisation");
  d->bed = H;
  d->lin_W = nullptr;  // the Jacobian depends on the bed
  return BSW_OK;
}

int bsw_step_begin(bsw_disc d, const bsw_params* p, double dt, const void* Wold, void* bold) {
  if (!d || !Wold || !bold || !(dt > 0)) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "bad argument");
  if (int rc = check_params(d, p)) return rc;
  StepBeginLaunch L{d, p, dt, Wold, bold};
  return dispatch(d, L);
}

int bsw_operator_apply(bsw_disc d, const bsw_params* p, double dt, const void* W, const void* bold, void* R) {
  if (!d || !W || !bold || !R || !(dt > 0)) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "bad argument");
  if (W == R || bold == R) return fail(d->mesh->ctx, BSW_E_ARG, "R must not alias W or b_old");
  if (int rc = check_params(d, p)) return rc;
  OpLaunch L{d, p, dt, W, bold, R};
  return dispatch(d, L);
}

int bsw_jacobian_linearize(bsw_disc d, const bsw_params* p, double dt, const void* W) {
  if (!d || !W || !(dt > 0)) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "bad argument");
  if (int rc = check_params(d, p)) return rc;
  bsw_ctx c = d->mesh->ctx;
  const size_t nb = (size_t)d->bs * d->bs * d->mesh->n_el;
  const size_t nf = (size_t)schur_numbers(d->mesh->dim, d->ref.np) * d->mesh->n_el;
  if (!d->blocks) {
    if (hipMalloc(&d->blocks, nf * sizeof(float)) != hipSuccess || hipMalloc(&d->blocks_raw, nb * d->wsize) != hipSuccess)
      return fail(c, BSW_E_OOM, "block-Jacobi storage");
  }
  d->lin_W = W;
  d->lin_prm = *p;
  d->lin_dt = dt;
  LinearizeLaunch L{d};
  return dispatch(d, L);
}

int bsw_jacobian_apply(bsw_disc d, const void* x, void* y) {
  if (!d || !x || !y) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "null argument");
  if (!d->lin_W) return fail(d->mesh->ctx, BSW_E_STATE, "jacobian_apply before jacobian_linearize");
  if (x == y) return fail(d->mesh->ctx, BSW_E_ARG, "x and y must not alias");
  JacApplyLaunch L{d, x, y};
  return dispatch(d, L);
}

int bsw_precond_apply(bsw_disc d, const void* x, void* y) {
  if (!d || !x || !y) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "null argument");
  if (!d->lin_W) return fail(d->mesh->ctx, BSW_E_STATE, "precond_apply before jacobian_linearize");
  if (x == y) return fail(d->mesh->ctx, BSW_E_ARG, "x and y must not alias");
  PrecLaunch L{d, x, y};
  return dispatch(d, L);
}

int bsw_jacobian_blocks(bsw_disc d, void* blocks) {
  if (!d || !blocks) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "null argument");
  if (!d->lin_W) return fail(d->mesh->ctx, BSW_E_STATE, "jacobian_blocks before jacobian_linearize");
  bsw_ctx c = d->mesh->ctx;
  BlocksLaunch L{d};
  if (int rc = dispatch(d, L)) return rc;
  const size_t bytes = (size_t)d->bs * d->bs * d->mesh->n_el * d->wsize;
  HIPCHK(c, hipMemcpyAsync(blocks, d->blocks_raw, bytes, hipMemcpyDeviceToDevice, c->stream));
  return BSW_OK;
}

int bsw_stage_update(bsw_disc d, const bsw_params* p, void* W, const void* dW, double alpha, double* norms_out) {
  if (!d || !W || !dW) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "null argument");
  bsw_ctx c = d->mesh->ctx;
  const int64_t n = bsw_state_len(d);
  const int nblk = red_blocks(n);
  if (int rc = ensure_part(d, (size_t)nblk * 4)) return rc;
  if (d->precision == BSW_FP64)
    hipLaunchKernelGGL((k_axpy_norms<double>), dim3(nblk), dim3(kRedThreads), 0, c->stream, (double*)W,
                       (const double*)dW, alpha, n, d->part);
  else
    hipLaunchKernelGGL((k_axpy_norms<float>), dim3(nblk), dim3(kRedThreads), 0, c->stream, (float*)W,
                       (const float*)dW, alpha, n, d->part);
  HIPCHK(c, hipGetLastError());
  if (!norms_out) return BSW_OK;
  const int ops[2] = {1, 1};
  if (int rc = finish(d, nblk, 2, ops, norms_out)) return rc;
  if (p) {
    double dg[4];
    if (int rc = bsw_diagnostics(d, p, W, dg)) return rc;
    norms_out[2] = dg[0];
    norms_out[3] = dg[1];
  } else {
    norms_out[2] = norms_out[3] = 0.0;
  }
  return BSW_OK;
}

int bsw_stage_update_noalloc(bsw_disc d, const bsw_params* p, void* W, const void* dW, double alpha,
                             double* norms_out) {
  if (!d || !W || !dW) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "null argument");
  bsw_ctx c = d->mesh->ctx;
  if (!c->scratch) return fail(c, BSW_E_STATE, "context has no scratch address");
  const int64_t n = bsw_state_len(d);
  const int nblk = red_blocks(n);
  const int nblk_diag = red_blocks(d->mesh->n_el);
  // partial slots this call needs: 2 per workgroup of the update, 4 per
  // workgroup of the diagnostics (the workgroup counts are capped at 1024)
  if ((int64_t)nblk * 2 > kScratchPartials || (int64_t)nblk_diag * 4 > kScratchPartials)
    return fail(c, BSW_E_ARG, "stage_update_noalloc: the reduction needs more than the " +
                                  std::to_string(kScratchPartials) + " partial sums of its scratch");
  double* part = c->scratch;
  double* dev_out = c->scratch + kScratchPartials;
  if (d->precision == BSW_FP64)
    hipLaunchKernelGGL((k_axpy_norms<double>), dim3(nblk), dim3(kRedThreads), 0, c->stream, (double*)W,
                       (const double*)dW, alpha, n, part);
  else
    hipLaunchKernelGGL((k_axpy_norms<float>), dim3(nblk), dim3(kRedThreads), 0, c->stream, (float*)W,
                       (const float*)dW, alpha, n, part);
  HIPCHK(c, hipGetLastError());
  if (!norms_out) return BSW_OK;
  const int ops2[2] = {1, 1};
  if (int rc = finish_into(d, part, dev_out, nblk, 2, ops2, norms_out)) return rc;
  if (p) {
    DiagLaunch L{d, p, W, nblk_diag, part};
    if (int rc = dispatch(d, L)) return rc;
    const int ops4[4] = {0, 0, 1, 2};
    double dg[4];
    if (int rc = finish_into(d, part, dev_out, nblk_diag, 4, ops4, dg)) return rc;
    norms_out[2] = dg[0];
    norms_out[3] = 100.0 * dg[1] / d->mesh->measure;
  } else {
    norms_out[2] = norms_out[3] = 0.0;
  }
  return BSW_OK;
}

int bsw_diagnostics(bsw_disc d, const bsw_params* p, const void* W, double* out4) {
  if (!d || !p || !W || !out4) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "null argument");
  const int nblk = red_blocks(d->mesh->n_el);
  if (int rc = ensure_part(d, (size_t)nblk * 4)) return rc;
  DiagLaunch L{d, p, W, nblk, d->part};
  if (int rc = dispatch(d, L)) return rc;
  const int ops[4] = {0, 0, 1, 2};
  if (int rc = finish(d, nblk, 4, ops, out4)) return rc;
  out4[1] = 100.0 * out4[1] / d->mesh->measure;
  return BSW_OK;
}

int bsw_norm2(bsw_disc d, const void* x, double* out) {
  if (!d || !x || !out) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "null argument");
  bsw_ctx c = d->mesh->ctx;
  const int64_t n = bsw_state_len(d);
  const int nblk = red_blocks(n);
  if (int rc = ensure_part(d, (size_t)nblk)) return rc;
  if (d->precision == BSW_FP64)
    hipLaunchKernelGGL((k_multidot<double>), dim3(nblk, 1), dim3(kRedThreads), 0, c->stream, (const double*)x,
                       (size_t)n, (const double*)x, n, 0, d->part);
  else
    hipLaunchKernelGGL((k_multidot<float>), dim3(nblk, 1), dim3(kRedThreads), 0, c->stream, (const float*)x,
                       (size_t)n, (const float*)x, n, 0, d->part);
  HIPCHK(c, hipGetLastError());
  const int ops[1] = {0};
  double s;
  if (int rc = finish(d, nblk, 1, ops, &s)) return rc;
  *out = std::sqrt(s);
  return BSW_OK;
}

int bsw_cfl_dt(bsw_disc d, const bsw_params* p, const void* W, double cfl, double* dt_out) {
  if (!d || !p || !W || !dt_out || !(cfl > 0)) return fail(d ? d->mesh->ctx : nullptr, BSW_E_ARG, "bad argument");
  double dg[4];
  if (int rc = bsw_diagnostics(d, p, W, dg)) return rc;
  *dt_out = cfl * d->mesh->hmin / dg[2];
  return BSW_OK;
}

}  // extern "C"

#include "bsw_batch.hpp"
