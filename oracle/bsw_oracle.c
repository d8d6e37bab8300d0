/*
 * Plain FP64 CPU oracle for the regularised-Bingham shallow-water DG method
 * (Fernandez, Lopez-Ordonez, Gonzalez-Andrade, arXiv 2301.11238).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * product path never does.  It shares no code, headers or tables with the
 * HIP library.
 *
 * What it computes (paper sections cited per function):
 *   - reference elements: normalised Legendre basis on [-1,1] (Sec. 5, modal
 *     expansion) and the orthonormal Dubiner basis on the unit triangle, with
 *     Gauss-Legendre and symmetric triangle quadrature;
 *   - pointwise maps U, F, Q, S, G (Sec. 3, Eqs. Uterm, Fterm, Qterm, Sterm,
 *     Gterm) and the regularised Bingham stress (Sec. 4);
 *   - HLL / central numerical fluxes (Sec. 5, Eq. HLLSolver);
 *   - element residuals of backward Euler (Sec. 5.1, Eq. WeakForm7);
 *   - their exact tangent (Appendix A, chain rule), the element diagonal
 *     blocks, a block-Jacobi preconditioned restarted GMRES for Eq. Newton
 *     and the Newton / time loop (Sec. 5.1, Sec. 6: at most 10 iterations);
 *   - diagnostics: mass and the active-region percentage (Sec. 6);
 *   - a variable bed H (Eq. Sterm, Sec. 5: H given at order m0 <= P) by
 *     nodal interpolation that is continuous across faces;
 *   - mixed orders m1, m2, m3 for h, u and E (Sec. 5): with bases ordered by
 *     total degree, field f lives in the span of its first N(m_f) modes and is
 *     tested with them; the remaining modes carry the trivial equations
 *     W = 0 (residual rows equal to the coefficient, identity Jacobian rows;
 *     the assembled blocks also drop their columns, so those modes stay
 *     exactly zero through Newton).
 *
 * Layout inside the oracle: per-element blocks W[e][f][i] (f = field,
 * i = mode).  Field order: h, u_1..u_d, then E_ab = d u_b / d x_a stored at
 * index 1 + d + b*d + a.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXP 4
#define MAXNP 15
#define MAXQ 16
#define MAXFQ 5
#define MAXNF 7
#define MAXNFC 3
#define MAXB (MAXNF * MAXNP)

/* ------------------------------------------------------------------ params */
typedef struct {
  double g, rho, alpha, eta, sigma0, gamma, beta;
  int32_t reg;      /* 1, 2, 3 (Sec. 4, Eqs. sigmaTwoA, sigmaTwoB, sigmaTwoC) */
  int32_t bc;       /* 1 wall, 2 Neumann, 3 Dirichlet (Sec. 5.2) */
  double dir[MAXNF]; /* Dirichlet exterior values (h, u..., E...) */
  int32_t jac_frozen; /* 1: the Jacobian holds S_L, S_R of the HLL flux fixed (Appendix A) */
  double dir_tag[3][MAXNF]; /* Dirichlet exterior values of boundary tags 1..3 */
} or_params;

typedef struct {
  int32_t kind;
  double a, b, c, d, x0, y0, r, L;
} or_ic;

/* Analytic bed: kind 0 flat, 1 a cos(kx x) cos(ky y) (1-D: a cos(kx x)),
 * 2 a exp(-|x - (x0, y0)|^2 / d); order = m0 (0: P). */
typedef struct {
  int32_t kind, order;
  double a, kx, ky, x0, y0, d;
} or_bed;

typedef struct {
  int32_t max_newton;   /* Sec. 6: at most 10 */
  int32_t gmres_m;
  int32_t gmres_max_restarts;
  double newton_tol;    /* ||dW||_inf <= tol (1 + ||W||_inf) */
  double gmres_rtol;
  double cfl, t_end;
  double dt_override;   /* > 0: use this dt instead of the CFL rule */
  int32_t max_steps;    /* < 0: all */
  double res_tol;       /* > 0: also stop when ||R||_2 <= res_tol ||b_old||_2 */
} or_solve_opts;

typedef struct {
  int32_t steps, newton_total, gmres_total, newton_max, capped;
  double dt, mass0, mass_end, max_mass_drift, active_pct, t_end;
} or_solve_stats;

/* -------------------------------------------------------- reference element */
typedef struct {
  int dim, P, np, nq, nfq, nfc, nf;
  double qx[MAXQ][2], qw[MAXQ];            /* volume rule on the reference element */
  double phi[MAXQ][MAXNP];                 /* basis at volume points */
  double dphi[MAXQ][MAXNP][2];             /* reference gradient at volume points */
  double fphi[MAXNFC][MAXFQ][MAXNP];       /* basis at face points */
  double fw[MAXFQ];                        /* face weights on [-1,1] (1-D: 1) */
  double ref_measure;
} or_ref;

typedef struct {
  int dim, n_el, n_vert;
  int *nbr, *nbr_face;   /* [n_el*nfc] */
  double *detJ;          /* [n_el] */
  double *dxi;           /* [n_el*4]: dxi_r/dx_a at [r*2+a] */
  double *normal;        /* [n_el*nfc*2] */
  double *flen;          /* [n_el*nfc] */
  double *xq;            /* [n_el*nq*2] physical volume points */
  double *vx;            /* [n_el*3*2] vertex coordinates */
  int8_t *fbc;           /* [n_el*nfc] boundary code of each local face: kind | tag << 2 */
  double total_measure, hmin;
} or_mesh;

typedef struct {
  or_ref ref;
  or_mesh mesh;
  double *bed;           /* [n_el*np] modal coefficients of the bed H; NULL = flat */
  int nmode[3];          /* modes used by h, u and E (orders m1, m2, m3) */
} or_disc;

/* 1 when row (f*np + i) of an element block is a mode above its field's order */
static int row_unused(const or_disc* D, int row) {
  int np = D->ref.np, f = row / np, i = row % np, dim = D->ref.dim;
  int nm = f == 0 ? D->nmode[0] : (f <= dim ? D->nmode[1] : D->nmode[2]);
  return i >= nm;
}

/* Legendre polynomial P_n and derivative by the three-term recursion. */
static void legendre(int n, double x, double* p, double* dp) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { *p = 1.0; *dp = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    double d2 = ((2.0 * k + 1.0) * (p1 + x * d1) - k * d0) / (k + 1.0);
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *p = p1; *dp = d1;
}

/* Gauss-Legendre nodes/weights on [-1,1] by Newton on P_n. */
static void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(n, z, &p, &dp);
      double dz = p / dp;
      z -= dz;
      if (fabs(dz) < 1e-17) break;
    }
    double p, dp;
    legendre(n, z, &p, &dp);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

/* Jacobi polynomial P_n^{(a,0)}(x) and derivative, standard recursion. */
static void jacobi_a0(int n, double a, double x, double* p, double* dp) {
  const double b = 0.0;
  double pm1 = 1.0, dm1 = 0.0;
  if (n == 0) { *p = 1.0; *dp = 0.0; return; }
  double pc = 0.5 * ((a + b + 2.0) * x + (a - b));
  double dc = 0.5 * (a + b + 2.0);
  for (int k = 2; k <= n; ++k) {
    double c1 = 2.0 * k * (k + a + b) * (2.0 * k + a + b - 2.0);
    double c2 = (2.0 * k + a + b - 1.0) * (a * a - b * b);
    double c3 = (2.0 * k + a + b - 2.0) * (2.0 * k + a + b - 1.0) * (2.0 * k + a + b);
    double c4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * (2.0 * k + a + b);
    double pn = ((c2 + c3 * x) * pc - c4 * pm1) / c1;
    double dn = (c3 * pc + (c2 + c3 * x) * dc - c4 * dm1) / c1;
    pm1 = pc; dm1 = dc; pc = pn; dc = dn;
  }
  *p = pc; *dp = dc;
}

/* Orthonormal Dubiner basis on T = {xi, eta >= 0, xi + eta <= 1}.
 * phi_{pq} = c_pq * L_p(x, y) * J_q^{(2p+1,0)}(b), with the homogenised
 * Legendre L_p(x, y) = y^p P_p(x / y), x = 2 xi + eta - 1, y = 1 - eta,
 * b = 2 eta - 1, c_pq = sqrt(2 (2p+1)(p+q+1)).  Modes ordered by total degree
 * n = p + q, then by q ascending. */
static void dubiner(int P, double xi, double eta, double* phi, double (*dphi)[2]) {
  double x = 2.0 * xi + eta - 1.0, y = 1.0 - eta, bb = 2.0 * eta - 1.0;
  double L[MAXP + 1], Lx[MAXP + 1], Ly[MAXP + 1];
  L[0] = 1.0; Lx[0] = 0.0; Ly[0] = 0.0;
  if (P >= 1) { L[1] = x; Lx[1] = 1.0; Ly[1] = 0.0; }
  for (int n = 1; n < P; ++n) {
    L[n + 1] = ((2.0 * n + 1.0) * x * L[n] - n * y * y * L[n - 1]) / (n + 1.0);
    Lx[n + 1] = ((2.0 * n + 1.0) * (L[n] + x * Lx[n]) - n * y * y * Lx[n - 1]) / (n + 1.0);
    Ly[n + 1] = ((2.0 * n + 1.0) * x * Ly[n] - n * (2.0 * y * L[n - 1] + y * y * Ly[n - 1])) / (n + 1.0);
  }
  int k = 0;
  for (int n = 0; n <= P; ++n) {
    for (int q = 0; q <= n; ++q) {
      int p = n - q;
      double c = sqrt(2.0 * (2.0 * p + 1.0) * (p + q + 1.0));
      double J, dJ;
      jacobi_a0(q, 2.0 * p + 1.0, bb, &J, &dJ);
      phi[k] = c * L[p] * J;
      if (dphi) {
        /* d/dxi: dx/dxi = 2 ; d/deta: dx/deta = 1, dy/deta = -1, db/deta = 2 */
        dphi[k][0] = c * 2.0 * Lx[p] * J;
        dphi[k][1] = c * ((Lx[p] - Ly[p]) * J + L[p] * 2.0 * dJ);
      }
      ++k;
    }
  }
}

static void legendre_basis(int P, double xi, double* phi, double (*dphi)[2]) {
  for (int i = 0; i <= P; ++i) {
    double p, dp;
    legendre(i, xi, &p, &dp);
    double s = sqrt((2.0 * i + 1.0) / 2.0);
    phi[i] = s * p;
    if (dphi) { dphi[i][0] = s * dp; dphi[i][1] = 0.0; }
  }
}

/* Symmetric triangle rules (weights normalised to sum 1 here, scaled by the
 * reference area 1/2 afterwards).  Orbits in barycentric coordinates. */
typedef struct { int n; double l[MAXQ][3]; double w[MAXQ]; } tri_rule;

static void tri_add_s3(tri_rule* r, double w) {
  r->l[r->n][0] = r->l[r->n][1] = r->l[r->n][2] = 1.0 / 3.0; r->w[r->n++] = w;
}
static void tri_add_s21(tri_rule* r, double a, double w) {
  double c = 1.0 - 2.0 * a;
  double L[3][3] = {{a, a, c}, {a, c, a}, {c, a, a}};
  for (int k = 0; k < 3; ++k) { memcpy(r->l[r->n], L[k], sizeof(L[k])); r->w[r->n++] = w; }
}
static void tri_add_s111(tri_rule* r, double a, double b, double w) {
  double c = 1.0 - a - b;
  double L[6][3] = {{a, b, c}, {b, a, c}, {a, c, b}, {c, a, b}, {b, c, a}, {c, b, a}};
  for (int k = 0; k < 6; ++k) { memcpy(r->l[r->n], L[k], sizeof(L[k])); r->w[r->n++] = w; }
}

static double fact(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }

/* 12-point degree-6 rule: orbit parameters x = (a1, w1, a2, w2, b, c, w3) are
 * refined to full double precision by Gauss-Newton on the monomial moments
 * int_T xi^i eta^j = i! j! / (i+j+2)!, i + j <= 6 (published starting values). */
static void tri12_build(const double* x, tri_rule* r) {
  r->n = 0;
  tri_add_s21(r, x[0], x[1]);
  tri_add_s21(r, x[2], x[3]);
  tri_add_s111(r, x[4], x[5], x[6]);
}
static void tri12_resid(const double* x, double* res) {
  tri_rule r; tri12_build(x, &r);
  int m = 0;
  for (int i = 0; i <= 6; ++i)
    for (int j = 0; i + j <= 6; ++j) {
      double s = 0.0;
      for (int k = 0; k < r.n; ++k) s += r.w[k] * pow(r.l[k][1], i) * pow(r.l[k][2], j);
      res[m++] = s - 2.0 * fact(i) * fact(j) / fact(i + j + 2);
    }
}
static void tri12_refine(double* x) {
  const int NE = 28, NU = 7;
  for (int it = 0; it < 6; ++it) {
    double r0[28], J[28][7];
    tri12_resid(x, r0);
    for (int u = 0; u < NU; ++u) {
      double xp[7], xm[7], rp[28], rm[28], h = 1e-6;
      memcpy(xp, x, sizeof(xp)); memcpy(xm, x, sizeof(xm));
      xp[u] += h; xm[u] -= h;
      tri12_resid(xp, rp); tri12_resid(xm, rm);
      for (int e = 0; e < NE; ++e) J[e][u] = (rp[e] - rm[e]) / (2 * h);
    }
    double A[7][7] = {{0}}, g[7] = {0};
    for (int u = 0; u < NU; ++u) {
      for (int v = 0; v < NU; ++v)
        for (int e = 0; e < NE; ++e) A[u][v] += J[e][u] * J[e][v];
      for (int e = 0; e < NE; ++e) g[u] -= J[e][u] * r0[e];
    }
    for (int k = 0; k < NU; ++k) { /* Gaussian elimination, partial pivoting */
      int pv = k;
      for (int i = k + 1; i < NU; ++i) if (fabs(A[i][k]) > fabs(A[pv][k])) pv = i;
      if (pv != k) {
        for (int j = 0; j < NU; ++j) { double t = A[k][j]; A[k][j] = A[pv][j]; A[pv][j] = t; }
        double t = g[k]; g[k] = g[pv]; g[pv] = t;
      }
      for (int i = k + 1; i < NU; ++i) {
        double l = A[i][k] / A[k][k];
        for (int j = k; j < NU; ++j) A[i][j] -= l * A[k][j];
        g[i] -= l * g[k];
      }
    }
    for (int k = NU - 1; k >= 0; --k) {
      double s = g[k];
      for (int j = k + 1; j < NU; ++j) s -= A[k][j] * g[j];
      g[k] = s / A[k][k];
    }
    for (int u = 0; u < NU; ++u) x[u] += g[u];
  }
}

static int tri_rule_for(int P, tri_rule* r) {
  r->n = 0;
  if (P == 1) {            /* 3 points, degree 2 */
    tri_add_s21(r, 1.0 / 6.0, 1.0 / 3.0);
  } else if (P == 2) {     /* 7 points, degree 5 (Radon) */
    double s15 = sqrt(15.0);
    tri_add_s3(r, 9.0 / 40.0);
    tri_add_s21(r, (6.0 - s15) / 21.0, (155.0 - s15) / 1200.0);
    tri_add_s21(r, (6.0 + s15) / 21.0, (155.0 + s15) / 1200.0);
  } else if (P == 3) {     /* 12 points, degree 6 (Dunavant) */
    double x[7] = {0.063089014491502, 0.050844906370207, 0.249286745170910,
                   0.116786275726379, 0.053145049844817, 0.310352451033784,
                   0.082851075618374};
    tri12_refine(x);
    tri12_build(x, r);
  } else {
    return -1;
  }
  return 0;
}

static int ref_build(or_ref* R, int dim, int P) {
  memset(R, 0, sizeof(*R));
  R->dim = dim; R->P = P;
  R->nf = 1 + dim + dim * dim;
  if (dim == 1) {
    if (P < 0 || P > MAXP) return -1;
    R->np = P + 1; R->nq = P + 1; R->nfq = 1; R->nfc = 2; R->ref_measure = 2.0;
    double x[MAXQ], w[MAXQ];
    gauss_legendre(R->nq, x, w);
    for (int q = 0; q < R->nq; ++q) {
      R->qx[q][0] = x[q]; R->qw[q] = w[q];
      legendre_basis(P, x[q], R->phi[q], R->dphi[q]);
    }
    legendre_basis(P, -1.0, R->fphi[0][0], NULL);
    legendre_basis(P, 1.0, R->fphi[1][0], NULL);
    R->fw[0] = 1.0;
  } else if (dim == 2) {
    if (P < 1 || P > 3) return -1;
    tri_rule tr;
    if (tri_rule_for(P, &tr)) return -1;
    R->np = (P + 1) * (P + 2) / 2; R->nq = tr.n; R->nfq = P + 1; R->nfc = 3;
    R->ref_measure = 0.5;
    for (int q = 0; q < tr.n; ++q) {
      R->qx[q][0] = tr.l[q][1]; R->qx[q][1] = tr.l[q][2];
      R->qw[q] = 0.5 * tr.w[q];
      dubiner(P, R->qx[q][0], R->qx[q][1], R->phi[q], R->dphi[q]);
    }
    double t[MAXFQ];
    gauss_legendre(R->nfq, t, R->fw);
    /* local face f runs from reference vertex f to vertex f+1 */
    const double V[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    for (int f = 0; f < 3; ++f)
      for (int r = 0; r < R->nfq; ++r) {
        double s = 0.5 * (t[r] + 1.0);
        const double* A = V[f]; const double* B = V[(f + 1) % 3];
        dubiner(P, A[0] + s * (B[0] - A[0]), A[1] + s * (B[1] - A[1]), R->fphi[f][r], NULL);
      }
  } else {
    return -1;
  }
  return 0;
}

/* ------------------------------------------------------------------- mesh */
typedef struct { int64_t key; int e, f; } face_key;
static int cmp_face_key(const void* a, const void* b) {
  int64_t ka = ((const face_key*)a)->key, kb = ((const face_key*)b)->key;
  return ka < kb ? -1 : (ka > kb ? 1 : 0);
}

static int mesh_build(or_disc* D, int dim, int n_vert, const double* xy, int n_el,
                      const int32_t* e2v) {
  or_mesh* M = &D->mesh; const or_ref* R = &D->ref;
  memset(M, 0, sizeof(*M));
  M->dim = dim; M->n_el = n_el; M->n_vert = n_vert;
  int nfc = R->nfc, nvpe = dim + 1;
  M->nbr = malloc(sizeof(int) * n_el * nfc);
  M->nbr_face = malloc(sizeof(int) * n_el * nfc);
  M->detJ = malloc(sizeof(double) * n_el);
  M->dxi = calloc((size_t)n_el * 4, sizeof(double));
  M->normal = calloc((size_t)n_el * nfc * 2, sizeof(double));
  M->flen = malloc(sizeof(double) * n_el * nfc);
  M->xq = calloc((size_t)n_el * R->nq * 2, sizeof(double));
  M->vx = calloc((size_t)n_el * 6, sizeof(double));
  M->fbc = calloc((size_t)n_el * nfc, sizeof(int8_t));
  M->total_measure = 0.0; M->hmin = 1e300;
  for (int e = 0; e < n_el; ++e) {
    const int32_t* v = e2v + (size_t)e * nvpe;
    if (dim == 1) {
      double x0 = xy[v[0]], x1 = xy[v[1]], L = x1 - x0;
      if (!(L > 0)) return -2;
      M->vx[e * 6 + 0] = x0; M->vx[e * 6 + 2] = x1;
      M->detJ[e] = 0.5 * L;
      M->dxi[e * 4 + 0] = 2.0 / L;
      M->normal[(e * nfc + 0) * 2] = -1.0; M->normal[(e * nfc + 1) * 2] = 1.0;
      M->flen[e * nfc + 0] = M->flen[e * nfc + 1] = 1.0;
      M->total_measure += L;
      if (L < M->hmin) M->hmin = L;
      for (int q = 0; q < R->nq; ++q) M->xq[(e * R->nq + q) * 2] = x0 + 0.5 * (R->qx[q][0] + 1.0) * L;
    } else {
      double X[3], Y[3];
      for (int k = 0; k < 3; ++k) { X[k] = xy[2 * v[k]]; Y[k] = xy[2 * v[k] + 1]; }
      for (int k = 0; k < 3; ++k) { M->vx[e * 6 + 2 * k] = X[k]; M->vx[e * 6 + 2 * k + 1] = Y[k]; }
      double a = X[1] - X[0], b = X[2] - X[0], c = Y[1] - Y[0], d = Y[2] - Y[0];
      double det = a * d - b * c;
      if (!(det > 0)) return -2;
      M->detJ[e] = det;
      /* [dxi/dx dxi/dy; deta/dx deta/dy] = inverse of [a b; c d] */
      M->dxi[e * 4 + 0] = d / det; M->dxi[e * 4 + 1] = -b / det;
      M->dxi[e * 4 + 2] = -c / det; M->dxi[e * 4 + 3] = a / det;
      double lmax = 0.0;
      for (int f = 0; f < 3; ++f) {
        int A = f, B = (f + 1) % 3;
        double ex = X[B] - X[A], ey = Y[B] - Y[A], L = sqrt(ex * ex + ey * ey);
        M->flen[e * nfc + f] = L;
        M->normal[(e * nfc + f) * 2 + 0] = ey / L;
        M->normal[(e * nfc + f) * 2 + 1] = -ex / L;
        if (L > lmax) lmax = L;
      }
      M->total_measure += 0.5 * det;
      double alt = det / lmax;
      if (alt < M->hmin) M->hmin = alt;
      for (int q = 0; q < R->nq; ++q) {
        M->xq[(e * R->nq + q) * 2 + 0] = X[0] + a * R->qx[q][0] + b * R->qx[q][1];
        M->xq[(e * R->nq + q) * 2 + 1] = Y[0] + c * R->qx[q][0] + d * R->qx[q][1];
      }
    }
  }
  /* face matching through sorted vertex keys */
  face_key* K = malloc(sizeof(face_key) * (size_t)n_el * nfc);
  for (int e = 0; e < n_el; ++e)
    for (int f = 0; f < nfc; ++f) {
      const int32_t* v = e2v + (size_t)e * nvpe;
      int64_t key;
      if (dim == 1) key = v[f];
      else {
        int64_t A = v[f], B = v[(f + 1) % 3];
        int64_t lo = A < B ? A : B, hi = A < B ? B : A;
        key = lo * (int64_t)n_vert + hi;
      }
      K[e * nfc + f].key = key; K[e * nfc + f].e = e; K[e * nfc + f].f = f;
      M->nbr[e * nfc + f] = -1; M->nbr_face[e * nfc + f] = -1;
    }
  qsort(K, (size_t)n_el * nfc, sizeof(face_key), cmp_face_key);
  int64_t n = (int64_t)n_el * nfc;
  for (int64_t i = 0; i < n;) {
    int64_t j = i + 1;
    while (j < n && K[j].key == K[i].key) ++j;
    if (j - i == 2) {
      M->nbr[K[i].e * nfc + K[i].f] = K[i + 1].e; M->nbr_face[K[i].e * nfc + K[i].f] = K[i + 1].f;
      M->nbr[K[i + 1].e * nfc + K[i + 1].f] = K[i].e; M->nbr_face[K[i + 1].e * nfc + K[i + 1].f] = K[i].f;
    } else if (j - i > 2) {
      free(K); return -3;
    }
    i = j;
  }
  free(K);
  return 0;
}

/* --------------------------------------------------- constitutive law (Sec. 4) */
/* Paper's 1-D regularised Bingham terms sigma_B^k(E) and their derivatives
 * (Eqs. sigmaTwoA/AA, sigmaTwoB, sigmaTwoC; Appendix A).  Readings: the
 * two-argument smooth max is max_beta(a, b) = b + max_beta(a - b, 0), and the
 * bottom branch of the reg-2 derivative is 2*gamma. */
static double smax_beta(double x, double beta, double* dm) {
  double h = 0.5 / beta;
  if (x >= h) { *dm = 1.0; return x; }
  if (x <= -h) { *dm = 0.0; return 0.0; }
  *dm = beta * (x + h);
  return 0.5 * beta * (x + h) * (x + h);
}

double or_sigmaB_1d(int reg, double s0, double gam, double bet, double E, double* dsdE) {
  double aE = fabs(E), sg = (E > 0) - (E < 0);
  if (reg == 1) {
    double dm, m = smax_beta(gam * aE - s0, bet, &dm);
    double den = m + s0;
    *dsdE = 2.0 * s0 * gam / den - 2.0 * s0 * gam * gam * E * sg / (den * den) * dm;
    return 2.0 * s0 * gam * E / den;
  } else if (reg == 2) {
    double h = 0.5 / bet, y = gam * aE;
    if (y >= s0 + h) { *dsdE = 0.0; return 2.0 * s0 * sg; }
    if (y >= s0 - h) {
      double z = s0 - y + h;
      *dsdE = 2.0 * bet * gam * z;
      return sg * (2.0 * s0 - bet * z * z);
    }
    *dsdE = 2.0 * gam;
    return 2.0 * gam * E;
  } else {
    double t = tanh(gam * E);
    *dsdE = 2.0 * s0 * gam * (1.0 - t * t);
    return 2.0 * s0 * t;
  }
}

/* Reading of the regularisations in 2-D: sigma_B = psi_k(s) (D + tr(D) I),
 * s = ||D||_c / sqrt(2).  psi_k(s) = sigma_B^k(s) / (2 s) (the 1-D law at E = s
 * divided by 2s, extended continuously to s = 0).  Returns psi and
 * q = psi'(s) / (2 s). */
static void or_psi(const or_params* p, double s, double* psi, double* q) {
  double s0 = p->sigma0, gam = p->gamma, bet = p->beta;
  if (s0 == 0.0) { *psi = 0.0; *q = 0.0; return; } /* no yield stress: sigma_B = 0 */
  if (p->reg == 1) {
    double dm, m = smax_beta(gam * s - s0, bet, &dm);
    double den = s0 + m;
    *psi = s0 * gam / den;
    *q = (dm == 0.0) ? 0.0 : (-s0 * gam * gam * dm / (den * den)) / (2.0 * s);
  } else if (p->reg == 2) {
    double h = 0.5 / bet, y = gam * s;
    if (y >= s0 + h) { *psi = s0 / s; *q = -s0 / (2.0 * s * s * s); }
    else if (y >= s0 - h) {
      double z = s0 - y + h, num = 2.0 * s0 - bet * z * z;
      *psi = num / (2.0 * s);
      double dpsi = bet * z * gam / s - num / (2.0 * s * s);
      *q = dpsi / (2.0 * s);
    } else { *psi = gam; *q = 0.0; }
  } else {
    double x = gam * s;
    if (x == 0.0) *psi = s0 * gam;
    else *psi = s0 * gam * tanh(x) / x;
    double r; /* (x sech^2 x - tanh x) / x^3 */
    if (x < 1e-2) {
      double x2 = x * x;
      r = -2.0 / 3.0 + x2 * (8.0 / 15.0 + x2 * (-34.0 / 105.0 + x2 * (496.0 / 2835.0)));
    } else {
      double t = tanh(x);
      r = (x * (1.0 - t * t) - t) / (x * x * x);
    }
    *q = 0.5 * s0 * gam * gam * gam * r;
  }
}

/* sigma(E) = (2 eta + psi(s)) T, T = D + tr(D) I, D = (E + E^T)/2
 * (Eqs. DtensorE, binghamR, sigma1, reading of the regularisation).
 * E is given as Em[a][b] = d u_b / d x_a.  Optionally dsig[a][b][c][d] =
 * d sigma_ab / d E_cd. */
static void or_sigma(const or_params* p, int dim, double Em[2][2], double sig[2][2],
                     double dsig[2][2][2][2]) {
  double Dm[2][2], tr = 0.0, n2 = 0.0, T[2][2];
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) Dm[a][b] = 0.5 * (Em[a][b] + Em[b][a]);
  for (int a = 0; a < dim; ++a) tr += Dm[a][a];
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) { n2 += Dm[a][b] * Dm[a][b]; T[a][b] = Dm[a][b] + (a == b ? tr : 0.0); }
  n2 += tr * tr;
  double s = sqrt(0.5 * n2);
  double psi, q;
  or_psi(p, s, &psi, &q);
  double mu = 2.0 * p->eta + psi;
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) sig[a][b] = mu * T[a][b];
  if (dsig) {
    for (int a = 0; a < dim; ++a)
      for (int b = 0; b < dim; ++b)
        for (int c = 0; c < dim; ++c)
          for (int d = 0; d < dim; ++d) {
            double dT = 0.5 * ((a == c && b == d) + (a == d && b == c)) + ((a == b) && (c == d));
            dsig[a][b][c][d] = mu * dT + q * T[a][b] * T[c][d];
          }
  }
}

/* ---------------------------------------------------- pointwise maps (Sec. 3) */
typedef struct {
  double h, u[2], E[2][2];
} pstate;

static void unpack(int dim, const double* X, pstate* s) {
  memset(s, 0, sizeof(*s));
  s->h = X[0];
  for (int b = 0; b < dim; ++b) s->u[b] = X[1 + b];
  for (int b = 0; b < dim; ++b)
    for (int a = 0; a < dim; ++a) s->E[a][b] = X[1 + dim + b * dim + a];
}

/* U (Eq. Uterm), F_a (Eq. Fterm), Q_a (Eq. Qterm), S (Eq. Sterm):
 * outputs over the 1+dim balance equations.  dH is the bed gradient at the
 * point (NULL: flat bed). */
static void pointwise(const or_params* p, int dim, const pstate* s, const double* dH, double* U,
                      double F[2][3], double Q[2][3], double* S) {
  double gc = p->g * cos(p->alpha), gs = p->g * sin(p->alpha);
  double sig[2][2];
  or_sigma(p, dim, (double(*)[2])s->E, sig, NULL);
  U[0] = s->h;
  for (int b = 0; b < dim; ++b) U[1 + b] = s->h * s->u[b];
  for (int a = 0; a < dim; ++a) {
    F[a][0] = s->h * s->u[a];
    Q[a][0] = 0.0;
    for (int b = 0; b < dim; ++b) {
      F[a][1 + b] = s->h * s->u[a] * s->u[b] + (a == b ? 0.5 * gc * s->h * s->h : 0.0);
      Q[a][1 + b] = s->h * sig[b][a] / p->rho;
    }
  }
  S[0] = 0.0;
  for (int b = 0; b < dim; ++b) {
    S[1 + b] = (b == 0) ? -gs * s->h : 0.0;
    if (dH) S[1 + b] -= gc * s->h * dH[b];
  }
}

/* Tangents of the same maps (Appendix A: dU/dV, dF/dV, dQ/dV, dQ/dE, dS/dV). */
static void pointwise_tan(const or_params* p, int dim, const pstate* s, const pstate* ds,
                          const double* dH, double* dU, double dF[2][3], double dQ[2][3],
                          double* dS) {
  double gc = p->g * cos(p->alpha), gs = p->g * sin(p->alpha);
  double sig[2][2], dsig[2][2][2][2];
  or_sigma(p, dim, (double(*)[2])s->E, sig, dsig);
  dU[0] = ds->h;
  for (int b = 0; b < dim; ++b) dU[1 + b] = ds->h * s->u[b] + s->h * ds->u[b];
  for (int a = 0; a < dim; ++a) {
    dF[a][0] = ds->h * s->u[a] + s->h * ds->u[a];
    dQ[a][0] = 0.0;
    for (int b = 0; b < dim; ++b) {
      dF[a][1 + b] = ds->h * s->u[a] * s->u[b] + s->h * ds->u[a] * s->u[b] +
                     s->h * s->u[a] * ds->u[b] + (a == b ? gc * s->h * ds->h : 0.0);
      double dsg = 0.0;
      for (int c = 0; c < dim; ++c)
        for (int d = 0; d < dim; ++d) dsg += dsig[b][a][c][d] * ds->E[c][d];
      dQ[a][1 + b] = (ds->h * sig[b][a] + s->h * dsg) / p->rho;
    }
  }
  dS[0] = 0.0;
  for (int b = 0; b < dim; ++b) {
    dS[1 + b] = (b == 0) ? -gs * ds->h : 0.0;
    if (dH) dS[1 + b] -= gc * ds->h * dH[b];
  }
}

/* Normal flux A(V; n) = sum_a F_a n_a and its tangent. */
static void normal_flux(const or_params* p, int dim, const pstate* s, const double* n,
                        double* A, double* U) {
  double gc = p->g * cos(p->alpha);
  double un = 0.0;
  for (int a = 0; a < dim; ++a) un += s->u[a] * n[a];
  A[0] = s->h * un;
  U[0] = s->h;
  for (int b = 0; b < dim; ++b) {
    A[1 + b] = s->h * s->u[b] * un + 0.5 * gc * s->h * s->h * n[b];
    U[1 + b] = s->h * s->u[b];
  }
}
static void normal_flux_tan(const or_params* p, int dim, const pstate* s, const pstate* ds,
                            const double* n, double* dA, double* dU) {
  double gc = p->g * cos(p->alpha);
  double un = 0.0, dun = 0.0;
  for (int a = 0; a < dim; ++a) { un += s->u[a] * n[a]; dun += ds->u[a] * n[a]; }
  dA[0] = ds->h * un + s->h * dun;
  dU[0] = ds->h;
  for (int b = 0; b < dim; ++b) {
    dA[1 + b] = ds->h * s->u[b] * un + s->h * ds->u[b] * un + s->h * s->u[b] * dun +
                gc * s->h * ds->h * n[b];
    dU[1 + b] = ds->h * s->u[b] + s->h * ds->u[b];
  }
}

/* HLL flux (Eq. HLLSolver) with wave speeds u_n -+ sqrt(g h) evaluated on
 * both sides.  When dm/dp are given, also returns the directional derivative
 * dF: exact (including the dependence of S_L, S_R), or with S_L, S_R held
 * fixed as the paper's Appendix A does (p->jac_frozen). */
static void or_hll(const or_params* p, int dim, const pstate* m, const pstate* pl,
                   const double* n, double* Fn, const pstate* dm, const pstate* dp, double* dFn) {
  int ne = 1 + dim;
  double Am[3], Um[3], Ap[3], Up[3];
  normal_flux(p, dim, m, n, Am, Um);
  normal_flux(p, dim, pl, n, Ap, Up);
  double unm = 0.0, unp = 0.0;
  for (int a = 0; a < dim; ++a) { unm += m->u[a] * n[a]; unp += pl->u[a] * n[a]; }
  double cm = sqrt(p->g * m->h), cp = sqrt(p->g * pl->h);
  double l1 = unm - cm, l2 = unp - cp, r1 = unm + cm, r2 = unp + cp;
  double SL = l1 <= l2 ? l1 : l2;
  double SR = r1 >= r2 ? r1 : r2;
  int branch = (SL >= 0.0) ? 0 : ((SR <= 0.0) ? 2 : 1);
  if (branch == 0) for (int k = 0; k < ne; ++k) Fn[k] = Am[k];
  else if (branch == 2) for (int k = 0; k < ne; ++k) Fn[k] = Ap[k];
  else
    for (int k = 0; k < ne; ++k)
      Fn[k] = (SR * Am[k] - SL * Ap[k] + SL * SR * (Up[k] - Um[k])) / (SR - SL);
  if (!dFn) return;
  double dAm[3], dUm[3], dAp[3], dUp[3];
  normal_flux_tan(p, dim, m, dm, n, dAm, dUm);
  normal_flux_tan(p, dim, pl, dp, n, dAp, dUp);
  if (branch == 0) { for (int k = 0; k < ne; ++k) dFn[k] = dAm[k]; return; }
  if (branch == 2) { for (int k = 0; k < ne; ++k) dFn[k] = dAp[k]; return; }
  double dunm = 0.0, dunp = 0.0;
  for (int a = 0; a < dim; ++a) { dunm += dm->u[a] * n[a]; dunp += dp->u[a] * n[a]; }
  double dcm = 0.5 * p->g * dm->h / cm, dcp = 0.5 * p->g * dp->h / cp;
  double dSL = l1 <= l2 ? (dunm - dcm) : (dunp - dcp);
  double dSR = r1 >= r2 ? (dunm + dcm) : (dunp + dcp);
  if (p->jac_frozen) dSL = dSR = 0.0;
  double den = SR - SL;
  for (int k = 0; k < ne; ++k) {
    double num = SR * Am[k] - SL * Ap[k] + SL * SR * (Up[k] - Um[k]);
    double dnum = dSR * Am[k] + SR * dAm[k] - dSL * Ap[k] - SL * dAp[k] +
                  (dSL * SR + SL * dSR) * (Up[k] - Um[k]) + SL * SR * (dUp[k] - dUm[k]);
    dFn[k] = dnum / den - num * (dSR - dSL) / (den * den);
  }
}

/* Mirror image of a state across a wall with unit normal n: the reflection
 * R = I - 2 n n^T maps u to R u and the velocity gradient E to R E R. */
static void mirror_state(int dim, const double* n, const pstate* in, pstate* out) {
  double Rm[2][2];
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) Rm[a][b] = (a == b) - 2.0 * n[a] * n[b];
  *out = *in;
  for (int a = 0; a < dim; ++a) {
    double s = 0.0;
    for (int b = 0; b < dim; ++b) s += Rm[a][b] * in->u[b];
    out->u[a] = s;
  }
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) {
      double s = 0.0;
      for (int c = 0; c < dim; ++c)
        for (int d = 0; d < dim; ++d) s += Rm[a][c] * in->E[c][d] * Rm[d][b];
      out->E[a][b] = s;
    }
}

/* Exterior state on a boundary face (Sec. 5.2, plus the mirror-wall reading:
 * h+ = h-, u+ = R u-, E+ = R E- R, so that the central fluxes give u.n = 0 and
 * zero tangential traction, and the HLL mass flux vanishes).  code = the
 * face's kind | tag << 2: kind 1 wall, 2 Neumann, 3 Dirichlet, 0 the
 * parameters' bc; a Dirichlet face takes the state of its tag (0: dir). */
static void bc_exterior(const or_params* p, int dim, const double* n, int code, const pstate* in,
                        pstate* out, const pstate* din, pstate* dout) {
  int kind = (code & 3) ? (code & 3) : p->bc, tag = code >> 2;
  if (kind == 1) {
    mirror_state(dim, n, in, out);
    if (din) mirror_state(dim, n, din, dout);
  } else if (kind == 2) { /* homogeneous Neumann: V+ = V-, E+ = E- */
    *out = *in;
    if (din) *dout = *din;
  } else { /* Dirichlet: prescribed exterior values */
    unpack(dim, tag ? p->dir_tag[tag - 1] : p->dir, out);
    if (din) memset(dout, 0, sizeof(*dout));
  }
}

/* --------------------------------------------------- element residual (Sec. 5) */
static void eval_fields(const or_ref* R, const double* phi, const double* We, double* X) {
  for (int f = 0; f < R->nf; ++f) {
    double s = 0.0;
    for (int i = 0; i < R->np; ++i) s += phi[i] * We[f * R->np + i];
    X[f] = s;
  }
}

/* Residual of Eq. WeakForm7 on element e (without -b_old; added by caller).
 * If vown is given, computes the directional derivative dR_e/dW . v instead,
 * where vown is v on element e and vnbr[f] (may be NULL = zero) is v on the
 * neighbour across local face f. */
static void element_eval(const or_disc* D, const or_params* p, double dt, const double* W,
                         int e, const double* const* vnbr, const double* vown, double* Re) {
  const or_ref* R = &D->ref; const or_mesh* M = &D->mesh;
  int dim = R->dim, np = R->np, nf = R->nf, nfc = R->nfc, nfq = R->nfq;
  int bs = nf * np;
  const double* We = W + (size_t)e * bs;
  int tan = (vown != NULL);
  for (int k = 0; k < bs; ++k) Re[k] = 0.0;
  double detJ = M->detJ[e];
  const double* dxi = M->dxi + e * 4;
  /* volume terms */
  for (int q = 0; q < R->nq; ++q) {
    double X[MAXNF], dX[MAXNF];
    eval_fields(R, R->phi[q], We, X);
    pstate s, ds;
    unpack(dim, X, &s);
    double U[3], F[2][3], Q[2][3], S[3];
    /* physical bed gradient dH/dx_a = sum_i H_i sum_r dphi_i/dxi_r dxi_r/dx_a */
    double dH[2] = {0.0, 0.0};
    if (D->bed) {
      const double* He = D->bed + (size_t)e * np;
      for (int a = 0; a < dim; ++a)
        for (int i = 0; i < np; ++i)
          for (int r = 0; r < dim; ++r) dH[a] += He[i] * R->dphi[q][i][r] * dxi[r * 2 + a];
    }
    const double* dHq = D->bed ? dH : NULL;
    if (tan) {
      eval_fields(R, R->phi[q], vown, dX);
      unpack(dim, dX, &ds);
      pointwise_tan(p, dim, &s, &ds, dHq, U, F, Q, S);
    } else {
      pointwise(p, dim, &s, dHq, U, F, Q, S);
    }
    const double* Xv = tan ? dX : X;   /* E and u enter linearly in R_E */
    double wq = R->qw[q] * detJ;
    for (int i = 0; i < np; ++i) {
      double phi_i = R->phi[q][i], dphi[2] = {0, 0};
      for (int a = 0; a < dim; ++a)
        for (int r = 0; r < dim; ++r) dphi[a] += R->dphi[q][i][r] * dxi[r * 2 + a];
      for (int f = 0; f <= dim; ++f) {
        double v = phi_i * (U[f] / dt - S[f]);
        for (int a = 0; a < dim; ++a) v -= dphi[a] * (F[a][f] - Q[a][f]);
        Re[f * np + i] += wq * v;
      }
      for (int b = 0; b < dim; ++b)
        for (int a = 0; a < dim; ++a) {
          int c = 1 + dim + b * dim + a;
          Re[c * np + i] += wq * (phi_i * Xv[c] + dphi[a] * Xv[1 + b]);
        }
    }
  }
  /* face terms */
  for (int fc = 0; fc < nfc; ++fc) {
    int nb = M->nbr[e * nfc + fc], nbf = M->nbr_face[e * nfc + fc];
    const double* n = M->normal + (e * nfc + fc) * 2;
    double half = (dim == 1) ? 1.0 : 0.5 * M->flen[e * nfc + fc];
    for (int r = 0; r < nfq; ++r) {
      double Xm[MAXNF], Xp[MAXNF], dXm[MAXNF], dXp[MAXNF];
      pstate sm, sp, dsm, dsp;
      eval_fields(R, R->fphi[fc][r], We, Xm);
      unpack(dim, Xm, &sm);
      if (tan) { eval_fields(R, R->fphi[fc][r], vown, dXm); unpack(dim, dXm, &dsm); }
      if (nb >= 0) {
        int rr = nfq - 1 - r;  /* shared edge is traversed in the opposite direction */
        eval_fields(R, R->fphi[nbf][rr], W + (size_t)nb * bs, Xp);
        unpack(dim, Xp, &sp);
        if (tan) {
          if (vnbr && vnbr[fc]) { eval_fields(R, R->fphi[nbf][rr], vnbr[fc], dXp); unpack(dim, dXp, &dsp); }
          else memset(&dsp, 0, sizeof(dsp));
        }
      } else {
        bc_exterior(p, dim, n, M->fbc[e * nfc + fc], &sm, &sp, tan ? &dsm : NULL, &dsp);
      }
      double wr = R->fw[r] * half;
      double Fn[3], Qn[3] = {0, 0, 0}, Gn[2][2];
      if (!tan) {
        or_hll(p, dim, &sm, &sp, n, Fn, NULL, NULL, NULL);
        double U[3], F[2][3], Qm[2][3], Qp[2][3], S[3];
        pointwise(p, dim, &sm, NULL, U, F, Qm, S);
        pointwise(p, dim, &sp, NULL, U, F, Qp, S);
        for (int f = 0; f <= dim; ++f)
          for (int a = 0; a < dim; ++a) Qn[f] += 0.5 * (Qm[a][f] + Qp[a][f]) * n[a];
        for (int a = 0; a < dim; ++a)
          for (int b = 0; b < dim; ++b) Gn[a][b] = 0.5 * (sm.u[b] + sp.u[b]) * n[a];
      } else {
        double Fdummy[3];
        or_hll(p, dim, &sm, &sp, n, Fdummy, &dsm, &dsp, Fn);
        double dU[3], dF[2][3], dQm[2][3], dQp[2][3], dS[3];
        pointwise_tan(p, dim, &sm, &dsm, NULL, dU, dF, dQm, dS);
        pointwise_tan(p, dim, &sp, &dsp, NULL, dU, dF, dQp, dS);
        for (int f = 0; f <= dim; ++f)
          for (int a = 0; a < dim; ++a) Qn[f] += 0.5 * (dQm[a][f] + dQp[a][f]) * n[a];
        for (int a = 0; a < dim; ++a)
          for (int b = 0; b < dim; ++b) Gn[a][b] = 0.5 * (dsm.u[b] + dsp.u[b]) * n[a];
      }
      for (int i = 0; i < np; ++i) {
        double ph = R->fphi[fc][r][i] * wr;
        for (int f = 0; f <= dim; ++f) Re[f * np + i] += ph * (Fn[f] - Qn[f]);
        for (int b = 0; b < dim; ++b)
          for (int a = 0; a < dim; ++a) Re[(1 + dim + b * dim + a) * np + i] -= ph * Gn[a][b];
      }
    }
  }
}

/* ------------------------------------------------------------ public API */
void* or_create(int dim, int P, int n_vert, const double* xy, int n_el, const int32_t* e2v,
                int* err) {
  or_disc* D = calloc(1, sizeof(or_disc));
  int rc = ref_build(&D->ref, dim, P);
  if (!rc) rc = mesh_build(D, dim, n_vert, xy, n_el, e2v);
  if (rc) { free(D); *err = rc; return NULL; }
  D->nmode[0] = D->nmode[1] = D->nmode[2] = D->ref.np;
  *err = 0;
  return D;
}

void or_destroy(void* h) {
  or_disc* D = h;
  if (!D) return;
  or_mesh* M = &D->mesh;
  free(M->nbr); free(M->nbr_face); free(M->detJ); free(M->dxi); free(M->normal);
  free(M->flen); free(M->xq); free(M->vx); free(M->fbc); free(D->bed); free(D);
}

int or_sizes(void* h, int* out) {
  or_disc* D = h;
  out[0] = D->ref.dim; out[1] = D->ref.P; out[2] = D->ref.np; out[3] = D->ref.nq;
  out[4] = D->ref.nfq; out[5] = D->ref.nfc; out[6] = D->ref.nf; out[7] = D->mesh.n_el;
  return 0;
}

/* reference tables, for pins: qx[nq*2], qw[nq], phi[nq*np], dphi[nq*np*2], fphi[nfc*nfq*np], fw[nfq] */
int or_ref_tables(void* h, double* qx, double* qw, double* phi, double* dphi, double* fphi,
                  double* fw) {
  or_ref* R = &((or_disc*)h)->ref;
  for (int q = 0; q < R->nq; ++q) {
    qx[2 * q] = R->qx[q][0]; qx[2 * q + 1] = R->qx[q][1]; qw[q] = R->qw[q];
    for (int i = 0; i < R->np; ++i) {
      phi[q * R->np + i] = R->phi[q][i];
      dphi[(q * R->np + i) * 2] = R->dphi[q][i][0];
      dphi[(q * R->np + i) * 2 + 1] = R->dphi[q][i][1];
    }
  }
  for (int f = 0; f < R->nfc; ++f)
    for (int r = 0; r < R->nfq; ++r)
      for (int i = 0; i < R->np; ++i) fphi[(f * R->nfq + r) * R->np + i] = R->fphi[f][r][i];
  for (int r = 0; r < R->nfq; ++r) fw[r] = R->fw[r];
  return 0;
}

/* basis evaluation at arbitrary reference points (pins) */
int or_basis(int dim, int P, int npts, const double* pts, double* phi, double* dphi) {
  int np = dim == 1 ? P + 1 : (P + 1) * (P + 2) / 2;
  for (int k = 0; k < npts; ++k) {
    double ph[MAXNP], dph[MAXNP][2];
    if (dim == 1) legendre_basis(P, pts[k], ph, dph);
    else dubiner(P, pts[2 * k], pts[2 * k + 1], ph, dph);
    for (int i = 0; i < np; ++i) {
      phi[k * np + i] = ph[i];
      if (dphi) { dphi[(k * np + i) * 2] = dph[i][0]; dphi[(k * np + i) * 2 + 1] = dph[i][1]; }
    }
  }
  return np;
}

/* mesh data, for pins: nbr, nbr_face [n_el*nfc], detJ [n_el], normal [n_el*nfc*2], flen, xq */
int or_mesh_data(void* h, int32_t* nbr, int32_t* nbrf, double* detJ, double* dxi, double* normal,
                 double* flen, double* xq, double* meas_hmin) {
  or_disc* D = h; or_mesh* M = &D->mesh; int nfc = D->ref.nfc;
  for (int k = 0; k < M->n_el * nfc; ++k) {
    nbr[k] = M->nbr[k]; nbrf[k] = M->nbr_face[k]; flen[k] = M->flen[k];
    normal[2 * k] = M->normal[2 * k]; normal[2 * k + 1] = M->normal[2 * k + 1];
  }
  for (int e = 0; e < M->n_el; ++e) {
    detJ[e] = M->detJ[e];
    for (int k = 0; k < 4; ++k) dxi[e * 4 + k] = M->dxi[e * 4 + k];
  }
  memcpy(xq, M->xq, sizeof(double) * (size_t)M->n_el * D->ref.nq * 2);
  meas_hmin[0] = M->total_measure; meas_hmin[1] = M->hmin;
  return 0;
}

/* b_old = (1/dt) <phi, U(W_old)> (first term of Eq. WeakForm7) */
int or_step_begin(void* h, const or_params* p, double dt, const double* Wold, double* bold) {
  or_disc* D = h; or_ref* R = &D->ref; or_mesh* M = &D->mesh;
  int dim = R->dim, np = R->np, bs = R->nf * np;
  (void)p;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < M->n_el; ++e) {
    double* b = bold + (size_t)e * bs;
    for (int k = 0; k < bs; ++k) b[k] = 0.0;
    for (int q = 0; q < R->nq; ++q) {
      double X[MAXNF]; pstate s;
      eval_fields(R, R->phi[q], Wold + (size_t)e * bs, X);
      unpack(dim, X, &s);
      double U[3]; U[0] = s.h;
      for (int c = 0; c < dim; ++c) U[1 + c] = s.h * s.u[c];
      double wq = R->qw[q] * M->detJ[e];
      for (int f = 0; f <= dim; ++f)
        for (int i = 0; i < np; ++i) b[f * np + i] += wq * R->phi[q][i] * U[f] / dt;
    }
  }
  return 0;
}

/* R(W) of Eq. WeakForm7 for every element */
int or_residual(void* h, const or_params* p, double dt, const double* W, const double* bold,
                double* Rout) {
  or_disc* D = h; int bs = D->ref.nf * D->ref.np, dim = D->ref.dim, np = D->ref.np;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < D->mesh.n_el; ++e) {
    double* Re = Rout + (size_t)e * bs;
    element_eval(D, p, dt, W, e, NULL, NULL, Re);
    for (int f = 0; f <= dim; ++f)
      for (int i = 0; i < np; ++i) Re[f * np + i] -= bold[(size_t)e * bs + f * np + i];
    for (int k = 0; k < bs; ++k)
      if (row_unused(D, k)) Re[k] = W[(size_t)e * bs + k];
  }
  return 0;
}

/* y = (dR/dW)(W) x, exact directional derivative (Appendix A) */
int or_jac_apply(void* h, const or_params* p, double dt, const double* W, const double* x,
                 double* y) {
  or_disc* D = h; int bs = D->ref.nf * D->ref.np;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < D->mesh.n_el; ++e) {
    const double* vn[MAXNFC] = {NULL, NULL, NULL};
    for (int f = 0; f < D->ref.nfc; ++f) {
      int nb = D->mesh.nbr[e * D->ref.nfc + f];
      if (nb >= 0) vn[f] = x + (size_t)nb * bs;
    }
    element_eval(D, p, dt, W, e, vn, x + (size_t)e * bs, y + (size_t)e * bs);
    for (int k = 0; k < bs; ++k)
      if (row_unused(D, k)) y[(size_t)e * bs + k] = x[(size_t)e * bs + k];
  }
  return 0;
}

/* diagonal blocks dR_e/dW_e, stored row-major [e][row][col] */
int or_jac_blocks(void* h, const or_params* p, double dt, const double* W, double* blocks) {
  or_disc* D = h; int bs = D->ref.nf * D->ref.np;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < D->mesh.n_el; ++e) {
    double v[MAXB], col[MAXB];
    double* B = blocks + (size_t)e * bs * bs;
    for (int j = 0; j < bs; ++j) {
      for (int k = 0; k < bs; ++k) v[k] = (k == j);
      element_eval(D, p, dt, W, e, NULL, v, col);
      for (int i = 0; i < bs; ++i)
        B[i * bs + j] = (row_unused(D, i) || row_unused(D, j)) ? (double)(i == j) : col[i];
    }
  }
  return 0;
}

/* face-coupling blocks dR_e/dW_nbr(e,f), stored [e][f][row][col]; zero on
 * boundary faces */
int or_jac_offdiag(void* h, const or_params* p, double dt, const double* W, double* blocks) {
  or_disc* D = h; int bs = D->ref.nf * D->ref.np, nfc = D->ref.nfc;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < D->mesh.n_el; ++e) {
    double v[MAXB], zero[MAXB], col[MAXB];
    for (int k = 0; k < bs; ++k) zero[k] = 0.0;
    for (int f = 0; f < nfc; ++f) {
      double* B = blocks + ((size_t)e * nfc + f) * bs * bs;
      if (D->mesh.nbr[e * nfc + f] < 0) { for (int k = 0; k < bs * bs; ++k) B[k] = 0.0; continue; }
      const double* vn[MAXNFC] = {NULL, NULL, NULL};
      vn[f] = v;
      for (int j = 0; j < bs; ++j) {
        for (int k = 0; k < bs; ++k) v[k] = (k == j);
        element_eval(D, p, dt, W, e, vn, zero, col);
        for (int i = 0; i < bs; ++i) B[i * bs + j] = (row_unused(D, i) || row_unused(D, j)) ? 0.0 : col[i];
      }
    }
  }
  return 0;
}

/* dense LU with partial pivoting, in place (row-major n x n) */
static int lu_factor(int n, double* A, int* piv) {
  for (int k = 0; k < n; ++k) {
    int pv = k;
    for (int i = k + 1; i < n; ++i) if (fabs(A[i * n + k]) > fabs(A[pv * n + k])) pv = i;
    piv[k] = pv;
    if (A[pv * n + k] == 0.0) return -1;
    if (pv != k)
      for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[pv * n + j]; A[pv * n + j] = t; }
    for (int i = k + 1; i < n; ++i) {
      double l = A[i * n + k] / A[k * n + k];
      A[i * n + k] = l;
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
    }
  }
  return 0;
}
static void lu_solve(int n, const double* A, const int* piv, double* b) {
  for (int k = 0; k < n; ++k) if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
  for (int i = 0; i < n; ++i) { double s = b[i]; for (int j = 0; j < i; ++j) s -= A[i * n + j] * b[j]; b[i] = s; }
  for (int i = n - 1; i >= 0; --i) { double s = b[i]; for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j]; b[i] = s / A[i * n + i]; }
}

static double dot(size_t n, const double* a, const double* b) {
  double s = 0.0; for (size_t i = 0; i < n; ++i) s += a[i] * b[i]; return s;
}

typedef struct {
  or_disc* D; const or_params* p; double dt; const double* W;
  double* lu; int* piv; int bs;
} lin_ctx;

static void apply_A(lin_ctx* c, const double* x, double* y) { or_jac_apply(c->D, c->p, c->dt, c->W, x, y); }
static void apply_Minv(lin_ctx* c, const double* x, double* y) {
  int bs = c->bs;
  memcpy(y, x, sizeof(double) * (size_t)c->D->mesh.n_el * bs);
#pragma omp parallel for schedule(static)
  for (int e = 0; e < c->D->mesh.n_el; ++e)
    lu_solve(bs, c->lu + (size_t)e * bs * bs, c->piv + (size_t)e * bs, y + (size_t)e * bs);
}

/* Right-preconditioned restarted GMRES(m), modified Gram-Schmidt + Givens.
 * Solves A x = b from x = 0 to ||b - A x|| <= rtol ||b||.  Returns iterations. */
static int gmres(lin_ctx* c, size_t n, const double* b, double* x, int m, double rtol,
                 int max_restarts, double* relres) {
  double* V = malloc(sizeof(double) * n * (m + 1));
  double* Z = malloc(sizeof(double) * n * m);
  double* w = malloc(sizeof(double) * n);
  double* r = malloc(sizeof(double) * n);
  double H[65][64], cs[64], sn[64], g[65];
  int its = 0;
  memset(x, 0, sizeof(double) * n);
  double bn = sqrt(dot(n, b, b));
  *relres = 0.0;
  if (bn == 0.0) { free(V); free(Z); free(w); free(r); return 0; }
  memcpy(r, b, sizeof(double) * n);
  double beta = bn;
  for (int rs = 0; rs <= max_restarts; ++rs) {
    for (size_t i = 0; i < n; ++i) V[i] = r[i] / beta;
    memset(g, 0, sizeof(g)); g[0] = beta;
    int j, done = 0;
    for (j = 0; j < m; ++j) {
      apply_Minv(c, V + j * n, Z + j * n);
      apply_A(c, Z + j * n, w);
      ++its;
      for (int i = 0; i <= j; ++i) {
        H[i][j] = dot(n, w, V + i * n);
        for (size_t k = 0; k < n; ++k) w[k] -= H[i][j] * V[i * n + k];
      }
      H[j + 1][j] = sqrt(dot(n, w, w));
      if (H[j + 1][j] != 0.0) for (size_t k = 0; k < n; ++k) V[(j + 1) * n + k] = w[k] / H[j + 1][j];
      for (int i = 0; i < j; ++i) {
        double t = cs[i] * H[i][j] + sn[i] * H[i + 1][j];
        H[i + 1][j] = -sn[i] * H[i][j] + cs[i] * H[i + 1][j];
        H[i][j] = t;
      }
      double den = sqrt(H[j][j] * H[j][j] + H[j + 1][j] * H[j + 1][j]);
      cs[j] = H[j][j] / den; sn[j] = H[j + 1][j] / den;
      H[j][j] = den; H[j + 1][j] = 0.0;
      g[j + 1] = -sn[j] * g[j]; g[j] = cs[j] * g[j];
      if (fabs(g[j + 1]) <= rtol * bn) { ++j; done = 1; break; }
    }
    double y[64];
    for (int i = j - 1; i >= 0; --i) {
      double s = g[i];
      for (int k = i + 1; k < j; ++k) s -= H[i][k] * y[k];
      y[i] = s / H[i][i];
    }
    for (int i = 0; i < j; ++i)
      for (size_t k = 0; k < n; ++k) x[k] += y[i] * Z[i * n + k];
    apply_A(c, x, w);
    for (size_t k = 0; k < n; ++k) r[k] = b[k] - w[k];
    beta = sqrt(dot(n, r, r));
    *relres = beta / bn;
    if (done || beta <= rtol * bn) break;
  }
  free(V); free(Z); free(w); free(r);
  return its;
}

/* One backward-Euler step by Newton (Eq. Newton, at most max_newton
 * iterations).  Converged when ||R||_2 <= res_tol ||b_old||_2 (res_tol > 0) for
 * the initial or an accepted residual.  Each iteration solves J dW = -R with
 * block-Jacobi GMRES and stops (converged, the update applied) when
 * ||dW||_inf <= newton_tol (1 + ||W||_inf); otherwise takes the largest step a
 * in {1, 1/2, ..., 1/64}
 * with ||R(W + a dW)|| <= (1 - 1e-4 a) ||R(W)|| (the smallest one if none does).
 * Returns the number of iterations; *conv = 1 converged, 0 capped, -1 non-finite. */
int or_newton_step(void* h, const or_params* p, double dt, double* W, const double* bold,
                   const or_solve_opts* o, int* conv, int* gmres_its) {
  or_disc* D = h;
  int bs = D->ref.nf * D->ref.np;
  size_t n = (size_t)D->mesh.n_el * bs;
  double* R = malloc(sizeof(double) * n);
  double* Rt = malloc(sizeof(double) * n);
  double* rhs = malloc(sizeof(double) * n);
  double* dW = malloc(sizeof(double) * n);
  double* Wt = malloc(sizeof(double) * n);
  double* lu = malloc(sizeof(double) * n * bs);
  int* piv = malloc(sizeof(int) * n);
  lin_ctx c = {D, p, dt, W, lu, piv, bs};
  int it = 0;
  *conv = 0; *gmres_its = 0;
  or_residual(D, p, dt, W, bold, R);
  double rn = sqrt(dot(n, R, R));
  const double rstop = o->res_tol > 0 ? o->res_tol * sqrt(dot(n, bold, bold)) : -1.0;
  if (isfinite(rn) && rn <= rstop) {
    *conv = 1;
    it = 0;
    goto done;
  }
  for (it = 1; it <= o->max_newton; ++it) {
    for (size_t k = 0; k < n; ++k) rhs[k] = -R[k];
    or_jac_blocks(D, p, dt, W, lu);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < D->mesh.n_el; ++e) lu_factor(bs, lu + (size_t)e * bs * bs, piv + (size_t)e * bs);
    double rr;
    *gmres_its += gmres(&c, n, rhs, dW, o->gmres_m, o->gmres_rtol, o->gmres_max_restarts, &rr);
    double dmax0 = 0.0, wmax0 = 0.0;
    for (size_t k = 0; k < n; ++k) {
      if (fabs(dW[k]) > dmax0) dmax0 = fabs(dW[k]);
      if (fabs(W[k]) > wmax0) wmax0 = fabs(W[k]);
    }
    if (isfinite(dmax0) && dmax0 <= o->newton_tol * (1.0 + wmax0)) {
      for (size_t k = 0; k < n; ++k) W[k] += dW[k];
      *conv = 1;
      break;
    }
    double a = 1.0, rnt = 0.0;
    for (;;) {
      for (size_t k = 0; k < n; ++k) Wt[k] = W[k] + a * dW[k];
      or_residual(D, p, dt, Wt, bold, Rt);
      rnt = sqrt(dot(n, Rt, Rt));
      if ((isfinite(rnt) && rnt <= (1.0 - 1e-4 * a) * rn) || a <= 1.0 / 64.0) break;
      a *= 0.5;
    }
    double dmax = 0.0, wmax = 0.0;
    int bad = !isfinite(rnt);
    for (size_t k = 0; k < n; ++k) {
      W[k] = Wt[k];
      if (!isfinite(W[k])) bad = 1;
      if (fabs(a * dW[k]) > dmax) dmax = fabs(a * dW[k]);
      if (fabs(W[k]) > wmax) wmax = fabs(W[k]);
    }
    memcpy(R, Rt, sizeof(double) * n);
    rn = rnt;
    (void)dmax; (void)wmax;
    if (bad) { *conv = -1; break; }
    if (rn <= rstop) { *conv = 1; break; }
  }
  if (it > o->max_newton) it = o->max_newton;
done:
  free(R); free(Rt); free(rhs); free(dW); free(Wt); free(lu); free(piv);
  return it;
}

/* L2 projection of an analytic initial condition (E = 0, Sec. 6). */
static void ic_value(const or_ic* ic, int dim, const double* x, double* h, double* u) {
  u[0] = u[1] = 0.0;
  double X = x[0], Y = dim == 2 ? x[1] : 0.0;
  switch (ic->kind) {
    case 0: *h = ic->a; u[0] = ic->b; u[1] = ic->c; break;
    case 1: *h = X < ic->x0 ? ic->a : ic->b; break;
    case 2: { double r2 = (X - ic->x0) * (X - ic->x0) + (dim == 2 ? (Y - ic->y0) * (Y - ic->y0) : 0.0);
              *h = ic->a + ic->b * exp(-r2 / ic->d); } break;
    case 3: { double r2 = (X - ic->x0) * (X - ic->x0) + (dim == 2 ? (Y - ic->y0) * (Y - ic->y0) : 0.0);
              *h = r2 < ic->r * ic->r ? ic->a : ic->b; } break;
    case 4: *h = ic->a; u[0] = ic->b * sin(M_PI * X / ic->L); break;
    case 5: *h = ic->a + ic->b * X; break;
    case 6: *h = ic->a; u[0] = ic->b * cos(M_PI * Y / ic->L); break;
    case 7: *h = ic->a;
            u[0] = ic->b * sin(M_PI * X / ic->L) * cos(M_PI * Y / ic->L);
            u[1] = -ic->b * cos(M_PI * X / ic->L) * sin(M_PI * Y / ic->L); break;
    case 8: *h = ic->a + ic->b * X; break;  /* free surface; the bed is subtracted below */
    default: *h = 1.0;
  }
}

/* Positivity reading for discontinuous initial depths: where the projected
 * depth falls below a tenth of the element mean at a volume or face point, the
 * non-constant depth modes are scaled so that the minimum becomes exactly a
 * tenth of the mean (the mean, hence the mass, is unchanged). */
static void ic_positivity(const or_ref* R, double* We) {
  int np = R->np;
  double mean = We[0] * R->phi[0][0];
  double mn = 1e300;
  for (int q = 0; q < R->nq; ++q) {
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += R->phi[q][i] * We[i];
    if (s < mn) mn = s;
  }
  for (int f = 0; f < R->nfc; ++f)
    for (int r = 0; r < R->nfq; ++r) {
      double s = 0.0;
      for (int i = 0; i < np; ++i) s += R->fphi[f][r][i] * We[i];
      if (s < mn) mn = s;
    }
  if (mean > 0.0 && mn < 0.1 * mean) {
    double theta = 0.9 * mean / (mean - mn);
    for (int i = 1; i < np; ++i) We[i] *= theta;
  }
}

int or_project_ic(void* h, const or_ic* ic, double* W) {
  or_disc* D = h; or_ref* R = &D->ref; or_mesh* M = &D->mesh;
  int dim = R->dim, np = R->np, bs = R->nf * np;
  for (int e = 0; e < M->n_el; ++e) {
    double* We = W + (size_t)e * bs;
    for (int k = 0; k < bs; ++k) We[k] = 0.0;
    for (int q = 0; q < R->nq; ++q) {
      double hv, u[2];
      ic_value(ic, dim, M->xq + (e * R->nq + q) * 2, &hv, u);
      for (int i = 0; i < np; ++i) {
        We[i] += R->qw[q] * R->phi[q][i] * hv;
        for (int b = 0; b < dim; ++b) We[(1 + b) * np + i] += R->qw[q] * R->phi[q][i] * u[b];
      }
    }
    if (ic->kind == 8) {
      /* h = a + b x - H: the linear surface is projected exactly, so h + H
       * equals it in coefficient space and h is as continuous as H */
      if (D->bed)
        for (int i = 0; i < np; ++i) We[i] -= D->bed[(size_t)e * np + i];
    }
    /* fields of lower order keep their first N(m_f) modes (the L2 projection
     * onto their space, the basis being orthonormal and hierarchical) */
    for (int k = 0; k < bs; ++k)
      if (row_unused(D, k)) We[k] = 0.0;
    if (ic->kind != 8) ic_positivity(R, We);
  }
  return 0;
}

/* ------------------------------------------------------------------ bed */
static double bed_value(const or_bed* b, int dim, double X, double Y) {
  switch (b->kind) {
    case 1: return b->a * cos(b->kx * X) * (dim == 2 ? cos(b->ky * Y) : 1.0);
    case 2: { double r2 = (X - b->x0) * (X - b->x0) + (dim == 2 ? (Y - b->y0) * (Y - b->y0) : 0.0);
              return b->a * exp(-r2 / b->d); }
    default: return 0.0;
  }
}

/* Interior Gauss-Lobatto points of order m on [-1, 1] (the roots of P_m'),
 * closed forms for m <= 4. */
static int lobatto_interior(int m, double* t) {
  switch (m) {
    case 1: return 0;
    case 2: t[0] = 0.0; return 1;
    case 3: t[0] = -1.0 / sqrt(5.0); t[1] = 1.0 / sqrt(5.0); return 2;
    case 4: t[0] = -sqrt(3.0 / 7.0); t[1] = 0.0; t[2] = sqrt(3.0 / 7.0); return 3;
  }
  return -1;
}

/* Interpolation nodes of order m on the reference element, chosen so that
 * the nodes on a face are the same physical points seen from both elements:
 * in 1-D the Gauss-Lobatto points; on the triangle the three vertices, the
 * interior Gauss-Lobatto points of every edge (symmetric about its midpoint)
 * and, for m = 3, the centroid.  Returns the node count. */
static int bed_nodes(int dim, int m, double (*xi)[2]) {
  double t[4];
  int ni = lobatto_interior(m, t), k = 0;
  if (ni < 0) return -1;
  if (dim == 1) {
    xi[k][0] = -1.0; xi[k++][1] = 0.0;
    for (int j = 0; j < ni; ++j) { xi[k][0] = t[j]; xi[k++][1] = 0.0; }
    xi[k][0] = 1.0; xi[k++][1] = 0.0;
    return k;
  }
  if (m > 3) return -1;
  const double V[3][2] = {{0, 0}, {1, 0}, {0, 1}};
  for (int v = 0; v < 3; ++v) { xi[k][0] = V[v][0]; xi[k++][1] = V[v][1]; }
  for (int f = 0; f < 3; ++f)
    for (int j = 0; j < ni; ++j) {
      double s = 0.5 * (t[j] + 1.0);
      const double* A = V[f]; const double* B = V[(f + 1) % 3];
      xi[k][0] = A[0] + s * (B[0] - A[0]); xi[k++][1] = A[1] + s * (B[1] - A[1]);
    }
  if (m == 3) { xi[k][0] = 1.0 / 3.0; xi[k++][1] = 1.0 / 3.0; }
  return k;
}

/* Bed of order m0 <= P (Sec. 5: H is given and projected at order m0; the
 * depth and the bed discretised alike): the interpolant of H at the order-m0
 * nodes, whose face traces agree between neighbours.  Both bases are
 * hierarchical by total degree, so the interpolant is spanned by the first
 * N(m0) modes; the Vandermonde system of those modes at the nodes gives its
 * coefficients and the higher modes are zero.  Out: H[e*np + i]. */
int or_bed_interpolate(void* h, const or_bed* bed, double* H) {
  or_disc* D = h; or_ref* R = &D->ref; or_mesh* M = &D->mesh;
  int dim = R->dim, np = R->np, m = bed->order > 0 ? bed->order : R->P;
  if (m > R->P || m < 1) return -1;
  double xi[MAXNP][2];
  int nn = bed_nodes(dim, m, xi);
  if (nn < 0) return -1;
  int nm = dim == 1 ? m + 1 : (m + 1) * (m + 2) / 2;
  if (nn != nm) return -1;
  double Vd[MAXNP * MAXNP]; int piv[MAXNP];
  for (int j = 0; j < nn; ++j) {
    double ph[MAXNP];
    if (dim == 1) legendre_basis(R->P, xi[j][0], ph, NULL);
    else dubiner(R->P, xi[j][0], xi[j][1], ph, NULL);
    for (int k = 0; k < nm; ++k) Vd[j * nm + k] = ph[k];
  }
  if (lu_factor(nm, Vd, piv)) return -1;
  for (int e = 0; e < M->n_el; ++e) {
    const double* v = M->vx + (size_t)e * 6;
    double c[MAXNP];
    for (int j = 0; j < nn; ++j) {
      double X, Y = 0.0;
      if (dim == 1) X = v[0] + 0.5 * (xi[j][0] + 1.0) * (v[2] - v[0]);
      else {
        X = v[0] + xi[j][0] * (v[2] - v[0]) + xi[j][1] * (v[4] - v[0]);
        Y = v[1] + xi[j][0] * (v[3] - v[1]) + xi[j][1] * (v[5] - v[1]);
      }
      c[j] = bed_value(bed, dim, X, Y);
    }
    lu_solve(nm, Vd, piv, c);
    for (int i = 0; i < np; ++i) H[(size_t)e * np + i] = i < nm ? c[i] : 0.0;
  }
  return 0;
}

/* Boundary codes per local face ([n_el*nfc], kind | tag << 2, Sec. 5.2);
 * interior faces are ignored; NULL: every boundary face takes the
 * parameters' bc. */
int or_set_boundary(void* h, const int8_t* codes) {
  or_disc* D = h; or_mesh* M = &D->mesh;
  size_t n = (size_t)M->n_el * D->ref.nfc;
  for (size_t k = 0; k < n; ++k) {
    int c = codes ? codes[k] : 0;
    if (c < 0 || c > 15) return -1;
    M->fbc[k] = (int8_t)(M->nbr[k] >= 0 ? 0 : c);
  }
  return 0;
}

/* Orders m1, m2, m3 of h, u and E (Sec. 5), each 0..P; P is the storage order. */
int or_set_orders(void* h, int m1, int m2, int m3) {
  or_disc* D = h;
  int m[3] = {m1, m2, m3};
  for (int k = 0; k < 3; ++k) {
    if (m[k] < 0 || m[k] > D->ref.P) return -1;
    D->nmode[k] = D->ref.dim == 1 ? m[k] + 1 : (m[k] + 1) * (m[k] + 2) / 2;
  }
  return 0;
}

/* Sets the bed used by the source term (a copy; NULL = flat). */
int or_set_bed(void* h, const double* H) {
  or_disc* D = h;
  free(D->bed); D->bed = NULL;
  if (!H) return 0;
  size_t n = (size_t)D->mesh.n_el * D->ref.np;
  D->bed = malloc(sizeof(double) * n);
  memcpy(D->bed, H, sizeof(double) * n);
  return 0;
}

/* mass = sum_e sum_q w_q h(x_q) ; active% = 100/|Omega| sum w_q H(s - sigma0/gamma) (Sec. 6) */
int or_diagnostics(void* h, const or_params* p, const double* W, double* out) {
  or_disc* D = h; or_ref* R = &D->ref; or_mesh* M = &D->mesh;
  int dim = R->dim, bs = R->nf * R->np;
  double mass = 0.0, act = 0.0, lam = 0.0, hmin = 1e300;
  for (int e = 0; e < M->n_el; ++e)
    for (int q = 0; q < R->nq; ++q) {
      double X[MAXNF]; pstate s;
      eval_fields(R, R->phi[q], W + (size_t)e * bs, X);
      unpack(dim, X, &s);
      double wq = R->qw[q] * M->detJ[e];
      mass += wq * s.h;
      double Dm[2][2], tr = 0.0, n2 = 0.0;
      for (int a = 0; a < dim; ++a) for (int b = 0; b < dim; ++b) Dm[a][b] = 0.5 * (s.E[a][b] + s.E[b][a]);
      for (int a = 0; a < dim; ++a) tr += Dm[a][a];
      for (int a = 0; a < dim; ++a) for (int b = 0; b < dim; ++b) n2 += Dm[a][b] * Dm[a][b];
      double sh = sqrt(0.5 * (n2 + tr * tr));
      if (sh - p->sigma0 / p->gamma >= 0.0) act += wq;
      double um = 0.0; for (int b = 0; b < dim; ++b) um += s.u[b] * s.u[b];
      double l = sqrt(um) + sqrt(p->g * (s.h > 0 ? s.h : 0.0));
      if (l > lam) lam = l;
      if (s.h < hmin) hmin = s.h;
    }
  out[0] = mass; out[1] = 100.0 * act / M->total_measure; out[2] = lam; out[3] = hmin;
  return 0;
}

/* field values at all volume quadrature points, [e][q][f] */
int or_eval_points(void* h, const double* W, double* vals) {
  or_disc* D = h; or_ref* R = &D->ref;
  int bs = R->nf * R->np;
  for (int e = 0; e < D->mesh.n_el; ++e)
    for (int q = 0; q < R->nq; ++q)
      eval_fields(R, R->phi[q], W + (size_t)e * bs, vals + ((size_t)e * R->nq + q) * R->nf);
  return 0;
}

/* Fixed time step from the initial state: dt = cfl * hmin / max(|u| + sqrt(g h)). */
double or_cfl_dt(void* h, const or_params* p, const double* W, double cfl) {
  double d[4];
  or_diagnostics(h, p, W, d);
  return cfl * ((or_disc*)h)->mesh.hmin / d[2];
}

/* Full solve: W holds the initial state on entry and the state at t_end on exit. */
int or_solve(void* h, const or_params* p, const or_solve_opts* o, double* W, or_solve_stats* st) {
  or_disc* D = h;
  int bs = D->ref.nf * D->ref.np;
  size_t n = (size_t)D->mesh.n_el * bs;
  double* bold = malloc(sizeof(double) * n);
  double diag[4];
  memset(st, 0, sizeof(*st));
  double dt = o->dt_override > 0 ? o->dt_override : or_cfl_dt(h, p, W, o->cfl);
  double nt = ceil(o->t_end / dt - 1e-12);
  if (!(nt <= 2.0e9)) return -1;
  int nsteps = (int)nt;
  if (nsteps < 1) nsteps = 1;
  if (o->max_steps >= 0 && nsteps > o->max_steps) nsteps = o->max_steps;
  or_diagnostics(h, p, W, diag);
  st->mass0 = diag[0]; st->dt = dt;
  double t = 0.0;
  for (int k = 1; k <= nsteps; ++k) {
    double dtk = (k < (int)nt) ? dt : o->t_end - (k - 1) * dt;
    or_step_begin(h, p, dtk, W, bold);
    int conv, gits;
    int its = or_newton_step(h, p, dtk, W, bold, o, &conv, &gits);
    st->newton_total += its; st->gmres_total += gits;
    if (its > st->newton_max) st->newton_max = its;
    if (conv != 1) st->capped++;
    if (conv < 0) break;
    or_diagnostics(h, p, W, diag);
    double drift = fabs(diag[0] - st->mass0) / st->mass0;
    if (drift > st->max_mass_drift) st->max_mass_drift = drift;
    t += dtk;
    st->steps = k;
  }
  or_diagnostics(h, p, W, diag);
  st->mass_end = diag[0]; st->active_pct = diag[1]; st->t_end = t;
  free(bold);
  return 0;
}

/* pointwise pins: stress and its derivative at one point (E as [E11,E21,E12,E22]) */
int or_point_sigma(const or_params* p, int dim, const double* Evec, double* sig, double* dsig) {
  double Em[2][2] = {{0, 0}, {0, 0}}, S[2][2], dS[2][2][2][2];
  for (int b = 0; b < dim; ++b) for (int a = 0; a < dim; ++a) Em[a][b] = Evec[b * dim + a];
  or_sigma(p, dim, Em, S, dS);
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) {
      sig[a * dim + b] = S[a][b];
      for (int c = 0; c < dim; ++c)
        for (int d = 0; d < dim; ++d)
          dsig[((a * dim + b) * dim + c) * dim + d] = dS[a][b][c][d];
    }
  return 0;
}

/* pointwise pins: HLL flux and directional derivative; states packed as X[nf] */
int or_point_hll(const or_params* p, int dim, const double* Xm, const double* Xp,
                 const double* n, const double* dXm, const double* dXp, double* F, double* dF) {
  pstate sm, sp, dsm, dsp;
  unpack(dim, Xm, &sm); unpack(dim, Xp, &sp);
  if (dXm) {
    unpack(dim, dXm, &dsm); unpack(dim, dXp, &dsp);
    double Fd[3];
    or_hll(p, dim, &sm, &sp, n, Fd, &dsm, &dsp, dF);
    for (int k = 0; k <= dim; ++k) F[k] = Fd[k];
  } else {
    or_hll(p, dim, &sm, &sp, n, F, NULL, NULL, NULL);
  }
  return 0;
}

/* pointwise pins: psi and q = psi'/(2s) */
int or_point_psi(const or_params* p, double s, double* out) {
  or_psi(p, s, &out[0], &out[1]);
  return 0;
}

/* wall exterior state (pins) */
int or_point_wall(const or_params* p, int dim, const double* n, const double* Xin, double* Xout) {
  pstate a, b;
  unpack(dim, Xin, &a);
  bc_exterior(p, dim, n, 0, &a, &b, NULL, NULL);
  Xout[0] = b.h;
  for (int k = 0; k < dim; ++k) Xout[1 + k] = b.u[k];
  for (int bb = 0; bb < dim; ++bb) for (int aa = 0; aa < dim; ++aa) Xout[1 + dim + bb * dim + aa] = b.E[aa][bb];
  return 0;
}
