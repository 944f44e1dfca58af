/*
 * FP64 CPU oracle for the narrow-band semi-Lagrangian level-set method of
 * S. Preda and M. Semplice, "Surface reconstruction from point cloud using a
 * semi-Lagrangian scheme with local interpolator" (arXiv:2410.22205).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header or
 * constant with the HIP library: every formula below is written out from the
 * paper's text, in double precision, one grid node at a time.
 *
 * Conventions (shared with the paper, Section 3):
 *   - uniform Cartesian grid, node (i,j[,k]) at x = lo + (i,j[,k]) * h,
 *     h the mesh width (the paper's Delta x);
 *   - storage in C order: 2D index i*n1 + j, 3D index (i*n1 + j)*n2 + k,
 *     axis 0 <-> x, axis 1 <-> y, axis 2 <-> z;
 *   - "centred finite differences" (Section 3, before 3.1) for every
 *     gradient, with first-order one-sided differences on the domain
 *     boundary (the paper is silent there).
 *
 * The OpenMP pragmas only split independent per-node loops (every update in
 * one time step reads the previous step only); they change no arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t dim;    /* 2 or 3 */
  int32_t n[3];   /* nodes per axis (n[2] ignored in 2D) */
  double lo[3];   /* coordinates of node 0 */
  double h;       /* mesh width */
} orc_grid;

typedef struct {
  double p;            /* exponent of the energy, Section 2 (only p = 1 used) */
  double delta;        /* weight of the curvature term, eq. (levelset:pde) */
  double gamma;        /* narrow-band half width, eq. (subgrid) */
  double beta;         /* inner radius of the cut-off, eq. (cutoff) */
  double grad_C;       /* C of the degenerate-gradient test, Section 3.1 */
  double grad_alpha;   /* alpha of the same test */
  double energy;       /* E_p(phi^n) in C^n_j; unused when p == 1 */
  int32_t reinit_every;  /* reinitialise after every K-th step */
  int32_t reinit_iters;  /* forward-Euler pseudo-time iterations */
  double reinit_dtau;    /* pseudo-time step */
  double interface_floor;/* lower bound of |grad| in the interface fix */
} orc_params;

/* ------------------------------------------------------------------ grid */

static int64_t orc_nodes(const orc_grid* g) {
  int64_t t = (int64_t)g->n[0] * g->n[1];
  return g->dim == 3 ? t * g->n[2] : t;
}

static int64_t orc_index(const orc_grid* g, const int c[3]) {
  if (g->dim == 3) return ((int64_t)c[0] * g->n[1] + c[1]) * g->n[2] + c[2];
  return (int64_t)c[0] * g->n[1] + c[1];
}

static void orc_coords(const orc_grid* g, int64_t idx, int c[3]) {
  if (g->dim == 3) {
    c[2] = (int)(idx % g->n[2]);
    idx /= g->n[2];
  } else {
    c[2] = 0;
  }
  c[1] = (int)(idx % g->n[1]);
  c[0] = (int)(idx / g->n[1]);
}

/* One component of the centred gradient of the nodal field f at node c. */
static double orc_diff(const double* f, const orc_grid* g, const int c[3], int a) {
  int cm[3] = {c[0], c[1], c[2]}, cp[3] = {c[0], c[1], c[2]};
  int has_m = c[a] > 0, has_p = c[a] < g->n[a] - 1;
  cm[a] -= 1;
  cp[a] += 1;
  if (has_m && has_p) return (f[orc_index(g, cp)] - f[orc_index(g, cm)]) / (2.0 * g->h);
  if (has_p) return (f[orc_index(g, cp)] - f[orc_index(g, c)]) / g->h;
  if (has_m) return (f[orc_index(g, c)] - f[orc_index(g, cm)]) / g->h;
  return 0.0;
}

void orc_gradient(const double* f, const orc_grid* g, int64_t idx, double* out) {
  int c[3];
  orc_coords(g, idx, c);
  for (int a = 0; a < 3; ++a) out[a] = a < g->dim ? orc_diff(f, g, c, a) : 0.0;
}

/* ---------------------------------------------------- cut-off, eq. (cutoff) */

double orc_cutoff(double phi, double beta, double gamma) {
  double a = fabs(phi);
  if (a <= beta) return 1.0;
  if (a <= gamma) {
    double gb = gamma - beta;
    return (a - gamma) * (a - gamma) * (2.0 * a + gamma - 3.0 * beta) / (gb * gb * gb);
  }
  return 0.0;
}

/* ------------------------------------------------------------ interpolation */

/* Cell that contains coordinate x along axis a and the local coordinate
 * theta = (x - x_i)/h in [0,1].  Points outside the grid are moved onto its
 * boundary (the paper is silent; the grid is meant to contain every foot). */
static void orc_locate(const orc_grid* g, int a, double x, int* i0, double* theta) {
  double u = (x - g->lo[a]) / g->h;
  double umax = (double)(g->n[a] - 1);
  if (u < 0.0) u = 0.0;
  if (u > umax) u = umax;
  int i = (int)floor(u);
  if (i > g->n[a] - 2) i = g->n[a] - 2;
  *i0 = i;
  *theta = u - (double)i;
}

/* Multilinear (Q1) interpolation, eq. (IQ1): the tensor-product degree-1
 * shape functions of the cell containing x, 2^dim terms. */
double orc_interp_q1(const double* f, const orc_grid* g, const double* x) {
  int i0[3] = {0, 0, 0};
  double t[3] = {0, 0, 0};
  for (int a = 0; a < g->dim; ++a) orc_locate(g, a, x[a], &i0[a], &t[a]);
  /* corner m has offset bit a of m along axis a */
  double v[8];
  int corners = 1 << g->dim;
  for (int m = 0; m < corners; ++m) {
    int c[3] = {i0[0], i0[1], i0[2]};
    for (int a = 0; a < g->dim; ++a) c[a] += (m >> a) & 1;
    v[m] = f[orc_index(g, c)];
  }
  /* The tensor product of linear interpolants, one axis at a time (last axis
   * first), each written as v0 + t (v1 - v0): equal to eq. (IQ1), and a cell
   * whose corners hold one value gives that value back exactly. */
  for (int a = g->dim - 1; a >= 0; --a) {
    int half = 1 << a;
    for (int m = 0; m < half; ++m) v[m] = v[m] + t[a] * (v[m + half] - v[m]);
  }
  return v[0];
}

/* One-dimensional third-order WENO interpolation on the cell [x_j, x_{j+1}]
 * (Section 3.2, n = 2).  v = (v_{j-1}, v_j, v_{j+1}, v_{j+2}), s = (x-x_j)/dx.
 *   P_L interpolates v on {x_{j-1}, x_j, x_{j+1}}, P_R on {x_j, x_{j+1}, x_{j+2}};
 *   C_L(x) = (x_{j+2}-x)/(3dx), C_R(x) = (x-x_{j-1})/(3dx)  (eq. ckgamma);
 *   I[P] = (1/dx^2) 4 a_2^2 with a_2 the coefficient of s^2 (eq. ind:1d);
 *   alpha_k = C_k/(I_k + eps)^2, eps = dx^2;  w_k = alpha_k / sum alpha;
 *   result = sum w_k P_k  (eq. IWENO).
 * The quadratics are written in Newton form about x_j and the sum as
 * P_R + w_L (P_L - P_R) (w_R = 1 - w_L): the same polynomials and the same
 * combination, evaluated so that a constant stencil returns its value
 * exactly (in the Lagrange form the basis functions sum to one only up to
 * rounding).  Foot points deep in the cut plateau then read exactly +-gamma.
 * parts (if not NULL) receives P_L, P_R, C_L, C_R, I_L, I_R, w_L, w_R. */
double orc_weno1d(const double* v, double s, double dx, double* parts) {
  double DL = v[0] - 2.0 * v[1] + v[2]; /* second differences: 2 a_2 */
  double DR = v[1] - 2.0 * v[2] + v[3];
  double PL = v[1] + 0.5 * s * (v[2] - v[0]) + 0.5 * s * s * DL;
  double PR = v[1] + s * (v[2] - v[1]) + 0.5 * s * (s - 1.0) * DR;
  double CL = (2.0 - s) / 3.0;
  double CR = (1.0 + s) / 3.0;
  double a2L = DL / 2.0;
  double a2R = DR / 2.0;
  double IL = 4.0 * a2L * a2L / (dx * dx);
  double IR = 4.0 * a2R * a2R / (dx * dx);
  double eps = dx * dx;
  double alL = CL / ((IL + eps) * (IL + eps));
  double alR = CR / ((IR + eps) * (IR + eps));
  double wL = alL / (alL + alR);
  double wR = 1.0 - wL;
  if (parts) {
    parts[0] = PL; parts[1] = PR; parts[2] = CL; parts[3] = CR;
    parts[4] = IL; parts[5] = IR; parts[6] = wL; parts[7] = wR;
  }
  return PR + wL * (PL - PR);
}

static int orc_clampi(int i, int n) { return i < 0 ? 0 : (i > n - 1 ? n - 1 : i); }

/* Tensor WENO interpolation (Section 3.2, last paragraphs): one-dimensional
 * WENO along the last axis first, then the previous one, then x.  Stencil
 * indices outside the grid repeat the boundary node. */
double orc_interp_weno(const double* f, const orc_grid* g, const double* x) {
  int i0[3] = {0, 0, 0};
  double t[3] = {0, 0, 0};
  for (int a = 0; a < g->dim; ++a) orc_locate(g, a, x[a], &i0[a], &t[a]);
  double h = g->h;
  if (g->dim == 2) {
    double wy[4];
    for (int a = 0; a < 4; ++a) {
      double v[4];
      int c[3] = {orc_clampi(i0[0] - 1 + a, g->n[0]), 0, 0};
      for (int b = 0; b < 4; ++b) {
        c[1] = orc_clampi(i0[1] - 1 + b, g->n[1]);
        v[b] = f[orc_index(g, c)];
      }
      wy[a] = orc_weno1d(v, t[1], h, NULL);
    }
    return orc_weno1d(wy, t[0], h, NULL);
  }
  double wx[4];
  for (int a = 0; a < 4; ++a) {
    double wy[4];
    for (int b = 0; b < 4; ++b) {
      double v[4];
      int c[3] = {orc_clampi(i0[0] - 1 + a, g->n[0]), orc_clampi(i0[1] - 1 + b, g->n[1]), 0};
      for (int e = 0; e < 4; ++e) {
        c[2] = orc_clampi(i0[2] - 1 + e, g->n[2]);
        v[e] = f[orc_index(g, c)];
      }
      wy[b] = orc_weno1d(v, t[2], h, NULL);
    }
    wx[a] = orc_weno1d(wy, t[1], h, NULL);
  }
  return orc_weno1d(wx, t[0], h, NULL);
}

double orc_interp(const double* f, const orc_grid* g, int kind, const double* x) {
  return kind == 0 ? orc_interp_q1(f, g, x) : orc_interp_weno(f, g, x);
}

/* ------------------------------------------------ semi-Lagrangian update */

/* Flags reported by orc_sl_node. */
#define ORC_FALLBACK 1   /* |grad phi| below C dt^alpha, eq. (SL:2) used */
#define ORC_FRAME0   2   /* 3D tangent frame regularised to (e1, e3) */

/* New value at band node idx, eqs. (SL2d)/(SL3d) with the cut-off factor of
 * Section 3.8 folded into C^n_j, followed by the cut of eq. (cut).
 * kind 0 = Q1, 1 = WENO. */
int orc_sl_node(const double* phi, const double* d, const orc_grid* g, const orc_params* P,
                double dt, int kind, int64_t idx, double* out) {
  int c[3];
  orc_coords(g, idx, c);
  double xj[3] = {0, 0, 0};
  for (int a = 0; a < g->dim; ++a) xj[a] = g->lo[a] + c[a] * g->h;
  double gp[3], gd[3];
  orc_gradient(phi, g, idx, gp);
  orc_gradient(d, g, idx, gd);
  double norm = sqrt(gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2]);
  int flags = 0;
  double val;
  if (norm < P->grad_C * pow(dt, P->grad_alpha)) {
    /* eq. (SL:2): mean of the interpolant over the first (face) neighbours,
     * which are grid nodes, so the interpolant returns the nodal values. */
    double sum = 0.0;
    int cnt = 0;
    for (int a = 0; a < g->dim; ++a) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int cn[3] = {c[0], c[1], c[2]};
        cn[a] += sgn;
        if (cn[a] < 0 || cn[a] > g->n[a] - 1) continue;
        sum += phi[orc_index(g, cn)];
        cnt += 1;
      }
    }
    val = sum / cnt;
    flags |= ORC_FALLBACK;
  } else {
    double C = orc_cutoff(phi[idx], P->beta, P->gamma);
    if (P->p != 1.0) C *= pow(d[idx] / P->energy, P->p - 1.0);
    double amp = sqrt(C * P->delta * d[idx] * dt / P->p);
    double base[3];
    for (int a = 0; a < 3; ++a) base[a] = xj[a] + C * dt * gd[a];
    if (g->dim == 2) {
      /* eq. (sigma2d): sigma = (d2 phi, -d1 phi)/|grad phi|, lambda = -1, +1 */
      double sg[2] = {gp[1] / norm, -gp[0] / norm};
      double sum = 0.0;
      for (int l = -1; l <= 1; l += 2) {
        double xs[3] = {base[0] + amp * sg[0] * l, base[1] + amp * sg[1] * l, 0.0};
        sum += orc_interp(phi, g, kind, xs);
      }
      val = sum / 2.0;
    } else {
      /* eq. (sigma3d) and the regularisation above it */
      double s = sqrt(gp[0] * gp[0] + gp[2] * gp[2]);
      double nu1[3], nu2[3];
      if (s != 0.0) {
        nu1[0] = -gp[2] / s; nu1[1] = 0.0; nu1[2] = gp[0] / s;
        nu2[0] = -gp[0] * gp[1] / s / norm;
        nu2[1] = s / norm;
        nu2[2] = -gp[1] * gp[2] / s / norm;
      } else {
        nu1[0] = 1.0; nu1[1] = 0.0; nu1[2] = 0.0;
        nu2[0] = 0.0; nu2[1] = 0.0; nu2[2] = 1.0;
        flags |= ORC_FRAME0;
      }
      double sum = 0.0;
      for (int l1 = -1; l1 <= 1; l1 += 2) {
        for (int l2 = -1; l2 <= 1; l2 += 2) {
          double xs[3];
          for (int a = 0; a < 3; ++a) xs[a] = base[a] + amp * (nu1[a] * l1 + nu2[a] * l2);
          sum += orc_interp(phi, g, kind, xs);
        }
      }
      val = sum / 4.0;
    }
  }
  if (val > P->gamma) val = P->gamma;
  if (val < -P->gamma) val = -P->gamma;
  *out = val;
  return flags;
}

/* Values at an arbitrary list of nodes (no band test). */
void orc_sl_nodes(const double* phi, const double* d, const orc_grid* g, const orc_params* P,
                  double dt, int kind, const int64_t* idx, int64_t m, double* out, int32_t* flags) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t e = 0; e < m; ++e) {
    int f = orc_sl_node(phi, d, g, P, dt, kind, idx[e], &out[e]);
    if (flags) flags[e] = f;
  }
}

/* One time step on the whole grid: band of eq. (subgrid) read as
 * |phi^n_j| < gamma, update inside it, every other node kept.
 * counts[0] += band size, counts[1] += fallbacks, counts[2] += frame
 * regularisations.  band (may be NULL) receives the 0/1 band mask. */
void orc_step(const double* phi, const double* d, const orc_grid* g, const orc_params* P,
              double dt, int kind, double* out, uint8_t* band, int64_t* counts) {
  int64_t N = orc_nodes(g);
  int64_t nb = 0, nf = 0, nr = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(+ : nb, nf, nr)
  for (int64_t j = 0; j < N; ++j) {
    int in = fabs(phi[j]) < P->gamma;
    if (band) band[j] = (uint8_t)in;
    if (!in) {
      out[j] = phi[j];
      continue;
    }
    int f = orc_sl_node(phi, d, g, P, dt, kind, j, &out[j]);
    nb += 1;
    nf += (f & ORC_FALLBACK) ? 1 : 0;
    nr += (f & ORC_FRAME0) ? 1 : 0;
  }
  if (counts) {
    counts[0] += nb;
    counts[1] += nf;
    counts[2] += nr;
  }
}

/* ----------------------------------------------------- reinitialisation */

static double orc_sign(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }

/* Constrained reinitialisation of Section 3.7 on the band of Section 3.8.
 * The paper gives the method only by reference; the reading used here:
 *   Gbar = band plus its face neighbours;
 *   interface set I = nodes of Gbar with a face neighbour of opposite (or
 *     zero) sign in phi~;
 *   one-step fix on I:  phi_j = phi~_j / max(|grad_c phi~_j|, floor);
 *   then reinit_iters forward-Euler steps of phi_tau + sign(phi~)(|grad phi|-1)
 *     = 0 on Gbar \ I with the first-order upwind (Godunov) gradient, I frozen;
 *   finally the cut of eq. (cut).
 * phi is overwritten.  counts[0] += |Gbar|, counts[1] += |I|. */
void orc_reinit(double* phi, const uint8_t* band, const orc_grid* g, const orc_params* P,
                int64_t* counts) {
  int64_t N = orc_nodes(g);
  uint8_t* gbar = (uint8_t*)calloc((size_t)N, 1);
  uint8_t* itf = (uint8_t*)calloc((size_t)N, 1);
  double* tilde = (double*)malloc((size_t)N * sizeof(double));
  double* cur = (double*)malloc((size_t)N * sizeof(double));
  double* nxt = (double*)malloc((size_t)N * sizeof(double));
  memcpy(tilde, phi, (size_t)N * sizeof(double));
  int64_t ng = 0, ni = 0;

#pragma omp parallel for reduction(+ : ng)
  for (int64_t j = 0; j < N; ++j) {
    int c[3];
    orc_coords(g, j, c);
    int in = band[j] != 0;
    for (int a = 0; a < g->dim && !in; ++a) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int cn[3] = {c[0], c[1], c[2]};
        cn[a] += sgn;
        if (cn[a] < 0 || cn[a] > g->n[a] - 1) continue;
        if (band[orc_index(g, cn)]) in = 1;
      }
    }
    gbar[j] = (uint8_t)in;
    ng += in;
  }

#pragma omp parallel for reduction(+ : ni)
  for (int64_t j = 0; j < N; ++j) {
    if (!gbar[j]) continue;
    int c[3];
    orc_coords(g, j, c);
    int is_if = 0;
    for (int a = 0; a < g->dim; ++a) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int cn[3] = {c[0], c[1], c[2]};
        cn[a] += sgn;
        if (cn[a] < 0 || cn[a] > g->n[a] - 1) continue;
        if (tilde[j] * tilde[orc_index(g, cn)] <= 0.0) is_if = 1;
      }
    }
    itf[j] = (uint8_t)is_if;
    ni += is_if;
  }

  memcpy(cur, tilde, (size_t)N * sizeof(double));
#pragma omp parallel for
  for (int64_t j = 0; j < N; ++j) {
    if (!itf[j]) continue;
    double gr[3];
    orc_gradient(tilde, g, j, gr);
    double nrm = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
    if (nrm < P->interface_floor) nrm = P->interface_floor;
    cur[j] = tilde[j] / nrm;
  }

  for (int it = 0; it < P->reinit_iters; ++it) {
    memcpy(nxt, cur, (size_t)N * sizeof(double));
#pragma omp parallel for
    for (int64_t j = 0; j < N; ++j) {
      if (!gbar[j] || itf[j]) continue;
      double S = orc_sign(tilde[j]);
      if (S == 0.0) continue;
      int c[3];
      orc_coords(g, j, c);
      double G2 = 0.0;
      for (int a = 0; a < g->dim; ++a) {
        int cm[3] = {c[0], c[1], c[2]}, cp[3] = {c[0], c[1], c[2]};
        cm[a] -= 1;
        cp[a] += 1;
        double Dm = c[a] > 0 ? (cur[j] - cur[orc_index(g, cm)]) / g->h : 0.0;
        double Dp = c[a] < g->n[a] - 1 ? (cur[orc_index(g, cp)] - cur[j]) / g->h : 0.0;
        double t1, t2;
        if (S > 0.0) {
          t1 = Dm > 0.0 ? Dm * Dm : 0.0;
          t2 = Dp < 0.0 ? Dp * Dp : 0.0;
        } else {
          t1 = Dm < 0.0 ? Dm * Dm : 0.0;
          t2 = Dp > 0.0 ? Dp * Dp : 0.0;
        }
        G2 += t1 > t2 ? t1 : t2;
      }
      nxt[j] = cur[j] - P->reinit_dtau * S * (sqrt(G2) - 1.0);
    }
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }

#pragma omp parallel for
  for (int64_t j = 0; j < N; ++j) {
    if (!gbar[j]) continue;
    double v = cur[j];
    if (v > P->gamma) v = P->gamma;
    if (v < -P->gamma) v = -P->gamma;
    phi[j] = v;
  }
  if (counts) {
    counts[0] += ng;
    counts[1] += ni;
  }
  free(gbar);
  free(itf);
  free(tilde);
  free(cur);
  free(nxt);
}

/* ----------------------------------------------------- Algorithm 1 loop */

/* n_steps passes of Algorithm 1, step 4, without the energy (p = 1):
 * band (a), update (c), and every reinit_every-th step the reinitialisation
 * on the band of that step and the cut (d).  step0 is the global index of the
 * first step, so that the reinitialisation phase survives a restart.
 * counts[0] = node updates, [1] fallbacks, [2] frame regularisations,
 * [3] reinitialisations, [4] sum |Gbar|, [5] sum |I|. */
void orc_run(double* phi, const double* d, const orc_grid* g, const orc_params* P, double dt,
             int kind, int64_t step0, int32_t n_steps, int64_t* counts) {
  int64_t N = orc_nodes(g);
  double* nxt = (double*)malloc((size_t)N * sizeof(double));
  uint8_t* band = (uint8_t*)malloc((size_t)N);
  int64_t local[6] = {0, 0, 0, 0, 0, 0};
  for (int32_t s = 0; s < n_steps; ++s) {
    orc_step(phi, d, g, P, dt, kind, nxt, band, local);
    if (P->reinit_every > 0 && (step0 + s + 1) % P->reinit_every == 0) {
      orc_reinit(nxt, band, g, P, &local[4]);
      local[3] += 1;
    }
    memcpy(phi, nxt, (size_t)N * sizeof(double));
  }
  if (counts) memcpy(counts, local, sizeof(local));
  free(nxt);
  free(band);
}

/* ------------------------------------------------------- initial data */

/* Closed-form signed distances used as phi^0, then the cut of eq. (cut).
 * kind 1: sphere (circle in 2D) centre args[0..2], radius args[3];
 * kind 2: torus with axis z, centre args[0..2], radii R = args[3], r = args[4]. */
void orc_init_phi(double* phi, const orc_grid* g, int kind, const double* args, double gamma) {
  int64_t N = orc_nodes(g);
#pragma omp parallel for
  for (int64_t j = 0; j < N; ++j) {
    int c[3];
    orc_coords(g, j, c);
    double x[3] = {0, 0, 0};
    for (int a = 0; a < g->dim; ++a) x[a] = g->lo[a] + c[a] * g->h - args[a];
    double v;
    if (kind == 1) {
      v = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) - args[3];
    } else {
      double rho = sqrt(x[0] * x[0] + x[1] * x[1]) - args[3];
      v = sqrt(rho * rho + x[2] * x[2]) - args[4];
    }
    if (v > gamma) v = gamma;
    if (v < -gamma) v = -gamma;
    phi[j] = v;
  }
}

/* ------------------------------------------------------ distance field */

/* d(x) = min_Q |x - Q| (Section 2), by brute force over all cloud points, at
 * every grid node.  pts is n_pts x dim, row major. */
void orc_distance_brute(const double* pts, int64_t n_pts, const orc_grid* g, double* d) {
  int64_t N = orc_nodes(g);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < N; ++j) {
    int c[3];
    orc_coords(g, j, c);
    double x[3] = {0, 0, 0};
    for (int a = 0; a < g->dim; ++a) x[a] = g->lo[a] + c[a] * g->h;
    double best = INFINITY;
    for (int64_t q = 0; q < n_pts; ++q) {
      double s = 0.0;
      for (int a = 0; a < g->dim; ++a) {
        double t = x[a] - pts[q * g->dim + a];
        s += t * t;
      }
      if (s < best) best = s;
    }
    d[j] = sqrt(best);
  }
}

/* ------------------------------------------------------ energy functional */

/* Section 3.5: E_p(phi) is approximated over the front cells, the cells of
 * the grid whose vertices do not all lie on one side of the front (a vertex
 * is inside when phi < 0), with |grad phi| = 1 assumed there.  This returns
 * the sum whose p-th root is E_p, the cells visited in index order:
 *  2D (eq. energyApprox, line form): the front crosses an edge where its two
 *     vertices lie on different sides, at the zero of the linear interpolant
 *     of phi along the edge; d there is the linear interpolant of d.  The
 *     integral over the segment between two crossings is taken by the
 *     trapezoidal rule, L (|d_1|^p + |d_2|^p) / 2.  A cell crossed on all four
 *     edges (reading: the paper names two points) gets two segments, paired
 *     so that the centre, where phi is the mean of the four vertex values,
 *     lies on the side of the vertex (i, j) when the two agree.
 *  3D (eq. energyApproxFiner): every front cell is split into R^3 subcells of
 *     side h' = h / R; phi and d at a subcell's centre are the trilinear
 *     interpolants of the cell's vertex values (reading: the reconstruction
 *     the paper leaves open), and the subcell adds |d|^p h'^2 when
 *     |phi| < (sqrt 3 / 2) h'. */
static double orc_lerp(double a, double b, double t) { return a + t * (b - a); }

static double orc_energy_2d_cell(const double* phi, const double* d, const orc_grid* g, int i,
                                 int j, double p) {
  /* corners in edge order: (i,j), (i+1,j), (i+1,j+1), (i,j+1) */
  const int ci[4] = {i, i + 1, i + 1, i}, cj[4] = {j, j, j + 1, j + 1};
  double f[4], e[4];
  int in[4], n_in = 0;
  for (int q = 0; q < 4; ++q) {
    int c[3] = {ci[q], cj[q], 0};
    int64_t k = orc_index(g, c);
    f[q] = phi[k];
    e[q] = d[k];
    in[q] = f[q] < 0.0;
    n_in += in[q];
  }
  if (n_in == 0 || n_in == 4) return 0.0;
  /* crossing on edge q (corner q to corner q + 1) */
  double px[4], py[4], pd[4];
  int has[4];
  for (int q = 0; q < 4; ++q) {
    int r = (q + 1) & 3;
    has[q] = in[q] != in[r];
    if (!has[q]) continue;
    double t = f[q] / (f[q] - f[r]);
    px[q] = g->lo[0] + g->h * orc_lerp(ci[q], ci[r], t);
    py[q] = g->lo[1] + g->h * orc_lerp(cj[q], cj[r], t);
    pd[q] = orc_lerp(e[q], e[r], t);
  }
  int pairs[2][2], n_seg = 0;
  if (has[0] && has[1] && has[2] && has[3]) {
    double centre = 0.25 * (f[0] + f[1] + f[2] + f[3]);
    if ((centre < 0.0) == in[0]) {
      /* the centre joins corner 0: segments cut off corners 1 and 3 */
      pairs[0][0] = 0; pairs[0][1] = 1;
      pairs[1][0] = 2; pairs[1][1] = 3;
    } else {
      /* segments cut off corners 0 and 2 */
      pairs[0][0] = 3; pairs[0][1] = 0;
      pairs[1][0] = 1; pairs[1][1] = 2;
    }
    n_seg = 2;
  } else {
    int a = -1, b = -1;
    for (int q = 0; q < 4; ++q)
      if (has[q]) {
        if (a < 0) a = q; else b = q;
      }
    pairs[0][0] = a;
    pairs[0][1] = b;
    n_seg = 1;
  }
  double s = 0.0;
  for (int m = 0; m < n_seg; ++m) {
    int a = pairs[m][0], b = pairs[m][1];
    double L = hypot(px[a] - px[b], py[a] - py[b]);
    s += L * 0.5 * (pow(fabs(pd[a]), p) + pow(fabs(pd[b]), p));
  }
  return s;
}

static double orc_energy_3d_cell(const double* phi, const double* d, const orc_grid* g, int i,
                                 int j, int k, double p, int R) {
  /* vertex values v[a][b][c] at (i + a, j + b, k + c) */
  double f[2][2][2], e[2][2][2];
  int n_in = 0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int c = 0; c < 2; ++c) {
        int cc[3] = {i + a, j + b, k + c};
        int64_t m = orc_index(g, cc);
        f[a][b][c] = phi[m];
        e[a][b][c] = d[m];
        n_in += phi[m] < 0.0;
      }
  if (n_in == 0 || n_in == 8) return 0.0;
  const double hs = g->h / R;
  const double lim = 0.5 * sqrt(3.0) * hs;
  double s = 0.0;
  for (int u = 0; u < R; ++u)
    for (int v = 0; v < R; ++v)
      for (int w = 0; w < R; ++w) {
        double tx = (u + 0.5) / R, ty = (v + 0.5) / R, tz = (w + 0.5) / R;
        /* trilinear: along x, then y, then z */
        double fy[2][2], ey[2][2];
        for (int b = 0; b < 2; ++b)
          for (int c = 0; c < 2; ++c) {
            fy[b][c] = orc_lerp(f[0][b][c], f[1][b][c], tx);
            ey[b][c] = orc_lerp(e[0][b][c], e[1][b][c], tx);
          }
        double fz0 = orc_lerp(fy[0][0], fy[1][0], ty), fz1 = orc_lerp(fy[0][1], fy[1][1], ty);
        double ez0 = orc_lerp(ey[0][0], ey[1][0], ty), ez1 = orc_lerp(ey[0][1], ey[1][1], ty);
        double fc = orc_lerp(fz0, fz1, tz), ec = orc_lerp(ez0, ez1, tz);
        if (fabs(fc) < lim) s += pow(fabs(ec), p) * hs * hs;
      }
  return s;
}

double orc_energy_sum(const double* phi, const double* d, const orc_grid* g, double p, int R) {
  double s = 0.0;
  if (g->dim == 2) {
    for (int i = 0; i + 1 < g->n[0]; ++i)
      for (int j = 0; j + 1 < g->n[1]; ++j) s += orc_energy_2d_cell(phi, d, g, i, j, p);
  } else {
    for (int i = 0; i + 1 < g->n[0]; ++i)
      for (int j = 0; j + 1 < g->n[1]; ++j)
        for (int k = 0; k + 1 < g->n[2]; ++k) s += orc_energy_3d_cell(phi, d, g, i, j, k, p, R);
  }
  return s;
}

/* ------------------------------------------------ initial data from the cloud */

/* Section 3.6: phi0 from the distance field d and a threshold gamma_S.
 *  1. External marking: the nodes on the boundary of the grid with
 *     d >= gamma_S are external; the marking then moves inwards through face
 *     neighbours, repeating sweeps along every Cartesian direction until no
 *     node changes, never entering a node with d < gamma_S (reading: the
 *     inward marking of Section 3.6 iterated to convergence, the serial
 *     result that the paper's parallel marking reproduces).
 *  2. phi0 = d - gamma_S on external nodes, a large value elsewhere.
 *  3. Fast sweeping (Zhao 2005): Gauss-Seidel sweeps in the 2^dim
 *     alternating orders of the first-order Godunov upwind discretisation
 *     of |grad u| = 1 recompute the internal values (external values
 *     fixed), until a full cycle changes nothing or max_cycles.
 *  4. The sign is reversed on internal nodes.
 * external[j] receives 1 for external nodes.  Returns the cycles used. */
static double orc_eik_update(const double* u, const orc_grid* g, const int c[3]) {
  double m[3];
  int n = 0;
  for (int a = 0; a < g->dim; ++a) {
    double best = INFINITY;
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      int cn[3] = {c[0], c[1], c[2]};
      cn[a] += sgn;
      if (cn[a] < 0 || cn[a] > g->n[a] - 1) continue;
      double v = u[orc_index(g, cn)];
      if (v < best) best = v;
    }
    if (best < INFINITY) m[n++] = best;
  }
  /* sort ascending */
  for (int i = 0; i < n; ++i)
    for (int k = i + 1; k < n; ++k)
      if (m[k] < m[i]) {
        double t = m[i];
        m[i] = m[k];
        m[k] = t;
      }
  const double h = g->h;
  if (n == 0) return INFINITY;
  double x = m[0] + h;
  if (n >= 2 && x > m[1]) {
    x = 0.5 * (m[0] + m[1] + sqrt(2.0 * h * h - (m[0] - m[1]) * (m[0] - m[1])));
    if (n >= 3 && x > m[2]) {
      double s = m[0] + m[1] + m[2];
      double q = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
      x = (s + sqrt(s * s - 3.0 * (q - h * h))) / 3.0;
    }
  }
  return x;
}

int orc_phi0_from_cloud(const double* d, const orc_grid* g, double gamma_s, int max_cycles,
                        double* phi, uint8_t* external) {
  const int64_t N = orc_nodes(g);
  const int dim = g->dim;
  const int n2 = dim == 3 ? g->n[2] : 1;
  memset(external, 0, (size_t)N);
  for (int64_t j = 0; j < N; ++j) {
    int c[3];
    orc_coords(g, j, c);
    int on_boundary = 0;
    for (int a = 0; a < dim; ++a) on_boundary |= c[a] == 0 || c[a] == g->n[a] - 1;
    if (on_boundary && d[j] >= gamma_s) external[j] = 1;
  }
  /* directional sweeps until no node changes */
  for (int changed = 1; changed;) {
    changed = 0;
    for (int a = 0; a < dim; ++a)
      for (int dir = -1; dir <= 1; dir += 2) {
        for (int i = 0; i < g->n[0]; ++i)
          for (int jj = 0; jj < g->n[1]; ++jj)
            for (int k = 0; k < n2; ++k) {
              int c[3] = {i, jj, k};
              /* visit along axis a in direction dir */
              if (dir < 0) c[a] = g->n[a] - 1 - c[a];
              int64_t idx = orc_index(g, c);
              if (external[idx] || d[idx] < gamma_s) continue;
              int cp[3] = {c[0], c[1], c[2]};
              cp[a] -= dir;
              if (cp[a] < 0 || cp[a] > g->n[a] - 1) continue;
              if (external[orc_index(g, cp)]) {
                external[idx] = 1;
                changed = 1;
              }
            }
      }
  }
  const double big = 1e30;
  for (int64_t j = 0; j < N; ++j) phi[j] = external[j] ? d[j] - gamma_s : big;
  /* fast sweeping over the internal nodes */
  int cycles = 0;
  for (; cycles < max_cycles; ++cycles) {
    int changed = 0;
    for (int o = 0; o < (1 << dim); ++o) {
      for (int i0 = 0; i0 < g->n[0]; ++i0)
        for (int j0 = 0; j0 < g->n[1]; ++j0)
          for (int k0 = 0; k0 < n2; ++k0) {
            int c[3] = {(o & 1) ? g->n[0] - 1 - i0 : i0, (o & 2) ? g->n[1] - 1 - j0 : j0,
                        dim == 3 ? ((o & 4) ? n2 - 1 - k0 : k0) : 0};
            int64_t idx = orc_index(g, c);
            if (external[idx]) continue;
            double x = orc_eik_update(phi, g, c);
            if (x < phi[idx]) {
              phi[idx] = x;
              changed = 1;
            }
          }
    }
    if (!changed) {
      ++cycles;
      break;
    }
  }
  for (int64_t j = 0; j < N; ++j)
    if (!external[j]) phi[j] = -phi[j];
  return cycles;
}

/* ------------------------------------------------ the paper's approximate d */

/* Section 3.4: d is set to its exact value (d_exact, the minimum over the
 * whole cloud) at every node of the box of 4 nodes per axis around each
 * cloud point (the two nodes on each side of the cell holding the point,
 * clamped to the grid), then the fast sweeping of orc_phi0_from_cloud's
 * step 3 (Zhao 2005) computes every other node from those.  Returns the
 * sweep cycles used. */
int orc_distance_approx(const double* pts, int64_t n_pts, const double* d_exact,
                        const orc_grid* g, int max_cycles, double* d, uint8_t* fixed) {
  const int64_t N = orc_nodes(g);
  const int dim = g->dim;
  const int n2 = dim == 3 ? g->n[2] : 1;
  memset(fixed, 0, (size_t)N);
  for (int64_t q = 0; q < n_pts; ++q) {
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
      int c = (int)floor((pts[q * dim + a] - g->lo[a]) / g->h);
      lo[a] = c - 1 < 0 ? 0 : c - 1;
      hi[a] = c + 2 > g->n[a] - 1 ? g->n[a] - 1 : c + 2;
    }
    for (int i = lo[0]; i <= hi[0]; ++i)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int k = lo[2]; k <= hi[2]; ++k) {
          int c[3] = {i, j, k};
          fixed[orc_index(g, c)] = 1;
        }
  }
  for (int64_t j = 0; j < N; ++j) d[j] = fixed[j] ? d_exact[j] : 1e30;
  int cycles = 0;
  for (; cycles < max_cycles; ++cycles) {
    int changed = 0;
    for (int o = 0; o < (1 << dim); ++o)
      for (int i0 = 0; i0 < g->n[0]; ++i0)
        for (int j0 = 0; j0 < g->n[1]; ++j0)
          for (int k0 = 0; k0 < n2; ++k0) {
            int c[3] = {(o & 1) ? g->n[0] - 1 - i0 : i0, (o & 2) ? g->n[1] - 1 - j0 : j0,
                        dim == 3 ? ((o & 4) ? n2 - 1 - k0 : k0) : 0};
            int64_t idx = orc_index(g, c);
            if (fixed[idx]) continue;
            double x = orc_eik_update(d, g, c);
            if (x < d[idx]) {
              d[idx] = x;
              changed = 1;
            }
          }
    if (!changed) {
      ++cycles;
      break;
    }
  }
  return cycles;
}

/* ------------------------------------------------ warm start of a finer run */

/* Section 4, after eq. (dxdt): every run after the first starts from the
 * steady state of the previous run, interpolated onto the run's own grid.
 * out[j] = I[f](x_j) at every node x_j of grid g, where f holds nodal values
 * on the coarser grid gf and I is the interpolator of Section 3.2 (kind 0:
 * IQ1, 1: tensor WENO); a node outside gf's box is moved onto it, as every
 * interpolation point is (orc_locate). */
void orc_resample(const double* f, const orc_grid* gf, int kind, const orc_grid* g, double* out) {
  const int64_t N = orc_nodes(g);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < N; ++j) {
    int c[3];
    orc_coords(g, j, c);
    double x[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < g->dim; ++a) x[a] = g->lo[a] + c[a] * g->h;
    out[j] = orc_interp(f, gf, kind, x);
  }
}

/* Worker threads of the OpenMP loops (n < 1: the runtime's default).  Used to
 * time the oracle on one core and on all of them. */
extern int omp_get_max_threads(void);
extern void omp_set_num_threads(int);
int orc_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}
