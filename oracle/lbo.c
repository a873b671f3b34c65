/*
 * lbo.c -- FP64 CPU oracle: colour-gradient lattice Boltzmann with
 * near-contact interactions.  TEST INFRASTRUCTURE ONLY (see lbo.h).
 *
 * One time step t -> t+1, in the order of the Materials and Methods section:
 *   1. rho^k = sum_i f_i^k, psi = (rho1 - rho2)/(rho1 + rho2)
 *   2. psi on wall rows copied from the adjacent fluid row (neutral wetting)
 *   3. G = 3 sum_i w_i c_i psi(x + c_i)   (second-order isotropic gradient)
 *      n = -G/|G|, delta_I = |G|/2
 *   4. NCI: h = first s in 1..floor(h_max) with psi(x + round(s n)) >= psi(x)
 *      (marching stops at a wall), A_h(h), F_rep = -A_h n delta_I (Eq. near_c).
 *      Continuous-NCI variant (nci_mode 1): psi sampled at x + s n by
 *      multilinear interpolation for s = 1..ceil(h_max), h refined to the
 *      linear crossing point between the last two samples, shifted A_h.
 *   5. F = F_body + F_rep
 *   6-7. f = f1 + f2, u = j/rho; BGK + exact-difference forcing + perturbation
 *   8. Latva-Kokko recolouring
 *   9. pull streaming with half-way bounce-back at wall rows
 * Density-ratio variant (rho_ratio > 0): component k has the equilibrium
 * E_i^k = rho_k phi_i^k + w_i rho_k (3 c.u + 4.5 (c.u)^2 - 1.5 u.u) with
 * phi_0^k = alpha_k and phi_i^k = (1 - alpha_k) w_i/(1 - w_0) otherwise, so
 * its sound speed is c_k^2 = (1 - alpha_k)/(3 (1 - w_0)); alpha_1 is given,
 * alpha_2 = 1 - gamma (1 - alpha_1) balances the pressures of the reference
 * densities rho_1^0 = 1, rho_2^0 = 1/gamma.  The collision relaxes the total
 * towards sum_k E^k; recolouring adds beta (rho1 rho2/rho^2) (rho1 phi_i^1 +
 * rho2 phi_i^2) cos(phi_i) to component 1; psi is normalised by the reference
 * densities, (rho1 - gamma rho2)/(rho1 + gamma rho2).
 * Geometry (lbo_set_geometry): a node-type mask on the periodic lattice.
 * Solid nodes reflect (half-way bounce-back) and carry psi = the w_i-weighted
 * mean of their non-solid neighbours (neutral wetting).  Inlet and outlet
 * nodes each have a feeder: their first fluid neighbour along -x, +x, -y, +y,
 * -z, +z.  After every collision an inlet takes the equilibrium at its
 * prescribed velocity and composition with the feeder's density (a velocity
 * inlet); an outlet takes the equilibrium at its prescribed density with the
 * feeder's velocity and composition (a pressure outlet).  Their fluid
 * neighbours then pull from them as from any node.  psi: inlets their
 * prescribed composition, outlets their feeder's.
 * Parity pins: tests/test_oracle_units.py and tests/test_oracle_physics.py.
 */
#include "lbo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* lattices smaller than this run on one thread: nodes are independent, so the
 * thread count never changes a result, and on small lattices the per-loop
 * synchronisation of a thread team costs more than the work */
#define LBO_PAR_MIN 16384

#define QMAX 27

struct lbo {
  lbo_params p;
  int Q, dim;
  int32_t c[QMAX][3];
  double w[QMAX];
  int32_t opp[QMAX];
  int64_t N, t;
  double *f1, *f2;   /* state at time t: [i][node]                 */
  double *g1, *g2;   /* post-collision scratch                     */
  double *psi;       /* order parameter (walls carry copied value) */
  uint8_t *type;     /* node types (lbo_set_geometry) or NULL       */
  double *in1, *in2, *inu; /* prescribed rho1, rho2 (N) and u (3N)  */
  int64_t *feeder;   /* fluid neighbour of each inlet/outlet (N)    */
};

/* ---- lattice (D2Q9 / D3Q27), weights by |c|^2 ----------------------- */
int lbo_lattice(int lattice, int32_t *c, double *w, int32_t *opp) {
  int Q = 0;
  if (lattice == LBO_D2Q9) {
    static const int v[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                                {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    static const double wt[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0};
    for (int i = 0; i < 9; ++i) {
      c[3 * i] = v[i][0]; c[3 * i + 1] = v[i][1]; c[3 * i + 2] = 0;
      w[i] = wt[v[i][0] * v[i][0] + v[i][1] * v[i][1]];
    }
    Q = 9;
  } else {
    static const double wt[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
    /* rest first, then all other velocities in z-major, y, x order */
    c[0] = c[1] = c[2] = 0; w[0] = wt[0]; Q = 1;
    for (int z = -1; z <= 1; ++z)
      for (int y = -1; y <= 1; ++y)
        for (int x = -1; x <= 1; ++x) {
          if (!x && !y && !z) continue;
          c[3 * Q] = x; c[3 * Q + 1] = y; c[3 * Q + 2] = z;
          w[Q] = wt[x * x + y * y + z * z];
          ++Q;
        }
  }
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j)
      if (c[3 * j] == -c[3 * i] && c[3 * j + 1] == -c[3 * i + 1] && c[3 * j + 2] == -c[3 * i + 2])
        opp[i] = j;
  return Q;
}

/* ---- equilibrium E_i(rho,u) = w_i rho [1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u] -- */
static double equilibrium_i(double w, const int32_t c[3], double rho, const double u[3]) {
  double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

void lbo_equilibrium(int lattice, double rho, const double u[3], double *feq) {
  int32_t c[QMAX][3], opp[QMAX];
  double w[QMAX];
  int Q = lbo_lattice(lattice, &c[0][0], w, opp);
  for (int i = 0; i < Q; ++i) feq[i] = equilibrium_i(w[i], c[i], rho, u);
}

/* ---- density-ratio variant: rest fractions and component equilibria ------ */
static int dr_on(const lbo_params *p) { return p->rho_ratio > 0; }
static void dr_alphas(const lbo_params *p, double w0, double *a1, double *a2) {
  if (!dr_on(p)) {
    *a1 = *a2 = w0;
    return;
  }
  *a1 = p->alpha1;
  *a2 = 1.0 - p->rho_ratio * (1.0 - p->alpha1);
}
/* phi_i^k of a direction with weight w (rest if c = 0) */
static double dr_phi(double alpha, double w, double w0, const int32_t c[3]) {
  int rest = c[0] == 0 && c[1] == 0 && c[2] == 0;
  return rest ? alpha : (1.0 - alpha) * w / (1.0 - w0);
}
static double equilibrium_k(double alpha, double w0, double w, const int32_t c[3], double rho,
                            const double u[3]) {
  double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return rho * dr_phi(alpha, w, w0, c) + w * rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

void lbo_equilibrium_k(int lattice, double alpha, double rho, const double u[3], double *feq) {
  int32_t c[QMAX][3], opp[QMAX];
  double w[QMAX];
  int Q = lbo_lattice(lattice, &c[0][0], w, opp);
  double w0 = 0;
  for (int i = 0; i < Q; ++i)
    if (!c[i][0] && !c[i][1] && !c[i][2]) w0 = w[i];
  for (int i = 0; i < Q; ++i) feq[i] = equilibrium_k(alpha, w0, w[i], c[i], rho, u);
}

/* ---- A_h: constant below h_min, (h_min/h)^3 decay up to h_max, 0 beyond -- */
double lbo_A_h(double h, double A, double h_min, double h_max) {
  if (h <= h_min) return A;
  if (h <= h_max) return A * (h_min / h) * (h_min / h) * (h_min / h);
  return 0.0;
}

double lbo_A_h_shifted(double h, double A, double h_min, double h_max) {
  if (h <= h_min) return A;
  if (h > h_max) return 0.0;
  double r = (h_min / h) * (h_min / h) * (h_min / h);
  double q = (h_min / h_max) * (h_min / h_max) * (h_min / h_max);
  return A * (r - q) / (1.0 - q);
}

/* ---- collision at one node (BGK + EDM + perturbation, then recolour) ---- */
static void collide(const lbo_params *p, int Q, int32_t (*c)[3], const double *w,
                    const double *f1, const double *f2, const double G[3],
                    const double F[3], double *o1, double *o2) {
  double rho1 = 0, rho2 = 0, j[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) {
    rho1 += f1[i];
    rho2 += f2[i];
  }
  double rho = rho1 + rho2;
  for (int i = 0; i < Q; ++i) {
    double fi = f1[i] + f2[i];
    for (int a = 0; a < 3; ++a) j[a] += c[i][a] * fi;
  }
  /* relaxation rate: one mixture tau, or the phase-weighted harmonic mean of
     the two components' relaxation times (viscosity-ratio variant) */
  double omega = 1.0 / p->tau;
  if (p->tau2 > 0) omega = (rho1 / rho) / p->tau + (rho2 / rho) / p->tau2;
  double u[3], uF[3];
  for (int a = 0; a < 3; ++a) {
    u[a] = j[a] / rho;
    uF[a] = u[a] + F[a] / rho; /* exact difference method: u + F dt / rho */
  }
  double g = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
  double Gh[3] = {0, 0, 0};
  if (g > 0)
    for (int a = 0; a < 3; ++a) Gh[a] = G[a] / g;
  double w0 = 0, al1, al2;
  for (int i = 0; i < Q; ++i)
    if (!c[i][0] && !c[i][1] && !c[i][2]) w0 = w[i];
  dr_alphas(p, w0, &al1, &al2);
  for (int i = 0; i < Q; ++i) {
    double fi = f1[i] + f2[i];
    double feq, feqF;
    if (dr_on(p)) {
      feq = equilibrium_k(al1, w0, w[i], c[i], rho1, u) + equilibrium_k(al2, w0, w[i], c[i], rho2, u);
      feqF = equilibrium_k(al1, w0, w[i], c[i], rho1, uF) + equilibrium_k(al2, w0, w[i], c[i], rho2, uF);
    } else {
      feq = equilibrium_i(w[i], c[i], rho, u);
      feqF = equilibrium_i(w[i], c[i], rho, uF);
    }
    double cG = c[i][0] * Gh[0] + c[i][1] * Gh[1] + c[i][2] * Gh[2];
    /* Omega1 (BGK) + forcing (EDM) + Omega2 (perturbation) */
    double pert = 0.5 * p->A_s * g * (w[i] * cG * cG - w[i] / 3.0);
    double fp = fi - (fi - feq) * omega + (feqF - feq) + pert;
    /* Omega3: recolouring with cos(phi_i) = c_i.G / (|c_i||G|) */
    double cnorm = sqrt((double)(c[i][0] * c[i][0] + c[i][1] * c[i][1] + c[i][2] * c[i][2]));
    double cosphi = (cnorm > 0) ? cG / cnorm : 0.0;
    double a1;
    if (dr_on(p))
      a1 = rho1 / rho * fp + p->beta * rho1 * rho2 / (rho * rho) *
                                 (rho1 * dr_phi(al1, w[i], w0, c[i]) + rho2 * dr_phi(al2, w[i], w0, c[i])) * cosphi;
    else
      a1 = rho1 / rho * fp + p->beta * rho1 * rho2 / rho * w[i] * cosphi;
    o1[i] = a1;
    o2[i] = fp - a1;
  }
}

void lbo_collide_node(const lbo_params *p, const double *f1, const double *f2,
                      const double G[3], const double F[3], double *out1, double *out2) {
  int32_t c[QMAX][3], opp[QMAX];
  double w[QMAX];
  int Q = lbo_lattice(p->lattice, &c[0][0], w, opp);
  collide(p, Q, c, w, f1, f2, G, F, out1, out2);
}

/* ---- geometry helpers ---------------------------------------------------- */
static int is_wall_y(const lbo_params *p, int y) {
  return p->walls_y && (y == 0 || y == p->ny - 1);
}
static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* neighbour of node (x,y,z) at offset (dx,dy,dz), periodic in every direction
 * (with walls the caller never leaves [0, ny-1] from a fluid row) */
static int64_t nb(const lbo_params *p, int x, int y, int z, int dx, int dy, int dz) {
  int xx = wrap(x + dx, p->nx), yy = wrap(y + dy, p->ny), zz = wrap(z + dz, p->nz);
  return xx + (int64_t)p->nx * (yy + (int64_t)p->ny * zz);
}

/* psi at a continuous position: multilinear interpolation of the node values
 * (lerp along x, then y, then z), wrapping along periodic axes; with walls
 * the stencil rows are clamped into the fluid rows [1, ny-2], i.e. psi is
 * extended beyond the fluid by the wall rows' copy rule. */
static double psi_at(const lbo_params *p, const double *psi, int dim, const double pos[3]) {
  int i0[3] = {0, 0, 0};
  double t[3] = {0, 0, 0};
  for (int a = 0; a < dim; ++a) {
    double f = floor(pos[a]);
    i0[a] = (int)f;
    t[a] = pos[a] - f;
  }
  double cz[2] = {0, 0};
  for (int kz = 0; kz < (dim == 3 ? 2 : 1); ++kz) {
    double cy[2];
    for (int ky = 0; ky < 2; ++ky) {
      double cx[2];
      for (int kx = 0; kx < 2; ++kx) {
        int xx = wrap(i0[0] + kx, p->nx);
        int yy = i0[1] + ky;
        if (p->walls_y) yy = yy < 1 ? 1 : (yy > p->ny - 2 ? p->ny - 2 : yy);
        else yy = wrap(yy, p->ny);
        int zz = dim == 3 ? wrap(i0[2] + kz, p->nz) : 0;
        cx[kx] = psi[xx + (int64_t)p->nx * (yy + (int64_t)p->ny * zz)];
      }
      cy[ky] = cx[0] + t[0] * (cx[1] - cx[0]);
    }
    cz[kz] = cy[0] + t[1] * (cy[1] - cy[0]);
  }
  return dim == 3 ? cz[0] + t[2] * (cz[1] - cz[0]) : cz[0];
}

/* gradient, NCI hit distance and F_rep at a fluid node; optionally the decision
 * margin (smallest |psi(y_s)-psi(x)| and distance of s*n to a rounding tie) */
static void node_nci(const lbo_params *p, int Q, int32_t (*c)[3], const double *w,
                     const double *psi, const uint8_t *type, int x, int y, int z, double G[3],
                     int32_t *hit, double Frep[3], double *margin) {
  int64_t self = x + (int64_t)p->nx * (y + (int64_t)p->ny * z);
  G[0] = G[1] = G[2] = 0;
  for (int i = 0; i < Q; ++i) {
    double ps = psi[nb(p, x, y, z, c[i][0], c[i][1], c[i][2])];
    for (int a = 0; a < 3; ++a) G[a] += 3.0 * w[i] * c[i][a] * ps;
  }
  double g = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
  Frep[0] = Frep[1] = Frep[2] = 0;
  *hit = 0;
  /* |G| enters the margin: whether the probe runs at all (G != 0) and the
   * direction n = -G/|G| it follows are ill-conditioned as |G| -> 0 */
  double mg = p->A_nci > 0 ? g : INFINITY;
  if (p->A_nci > 0 && g > 0 && p->nci_mode == 1) {
    /* continuous-NCI variant: first s with psi(x + s n) >= psi(x), h at the
     * linear crossing between samples s-1 and s (h = 1 for s = 1) */
    const int dim = p->lattice == LBO_D2Q9 ? 2 : 3;
    double n[3] = {-G[0] / g, -G[1] / g, -G[2] / g};
    int smax = (int)ceil(p->h_max);
    double prev = psi[self], h = 0;
    for (int s = 1; s <= smax; ++s) {
      double pos[3] = {x + s * n[0], y + s * n[1], z + s * n[2]};
      double ps = psi_at(p, psi, dim, pos);
      double d = fabs(ps - psi[self]);
      if (d < mg) mg = d;
      if (ps >= psi[self]) {
        *hit = s;
        h = s == 1 ? 1.0 : (s - 1) + (psi[self] - prev) / (ps - prev);
        break;
      }
      prev = ps;
    }
    if (*hit) {
      double Ah = lbo_A_h_shifted(h, p->A_nci, p->h_min, p->h_max);
      for (int a = 0; a < 3; ++a) Frep[a] = -Ah * n[a] * 0.5 * g;
    }
  } else if (p->A_nci > 0 && g > 0) {
    double n[3] = {-G[0] / g, -G[1] / g, -G[2] / g};
    int smax = (int)floor(p->h_max);
    for (int s = 1; s <= smax; ++s) {
      int off[3];
      for (int a = 0; a < 3; ++a) {
        double v = s * n[a];
        off[a] = (int)round(v); /* half away from zero */
        double tie = fabs(fabs(v - trunc(v)) - 0.5);
        if (tie < mg) mg = tie;
      }
      if (is_wall_y(p, y + off[1]) || (p->walls_y && (y + off[1] < 0 || y + off[1] >= p->ny)))
        break; /* the probe stops at a wall: no facing interface */
      if (type && type[nb(p, x, y, z, off[0], off[1], off[2])] != LBO_FLUID)
        break; /* ... and at any node that is not fluid */
      double py = psi[nb(p, x, y, z, off[0], off[1], off[2])];
      double d = fabs(py - psi[self]);
      if (d < mg) mg = d;
      if (py >= psi[self]) {
        *hit = s;
        break;
      }
    }
    if (*hit) {
      double Ah = lbo_A_h((double)*hit, p->A_nci, p->h_min, p->h_max);
      /* F_rep = -A_h n delta_I with delta_I = g/2, i.e. A_h G / 2 */
      for (int a = 0; a < 3; ++a) Frep[a] = -Ah * n[a] * 0.5 * g;
    }
  }
  if (margin) *margin = mg;
}

void lbo_node_nci(const lbo_params *p, const double *psi, int64_t node, double G[3],
                  int32_t *hit, double Frep[3]) {
  int32_t c[QMAX][3], opp[QMAX];
  double w[QMAX];
  int Q = lbo_lattice(p->lattice, &c[0][0], w, opp);
  int x = (int)(node % p->nx);
  int y = (int)((node / p->nx) % p->ny);
  int z = (int)(node / ((int64_t)p->nx * p->ny));
  node_nci(p, Q, c, w, psi, NULL, x, y, z, G, hit, Frep, NULL);
}

/* ---- handle ---------------------------------------------------------------- */
lbo *lbo_create(const lbo_params *p) {
  lbo *h = (lbo *)calloc(1, sizeof(lbo));
  h->p = *p;
  h->Q = lbo_lattice(p->lattice, &h->c[0][0], h->w, h->opp);
  h->dim = (p->lattice == LBO_D2Q9) ? 2 : 3;
  h->N = (int64_t)p->nx * p->ny * p->nz;
  size_t n = (size_t)h->Q * (size_t)h->N;
  h->f1 = (double *)calloc(n, sizeof(double));
  h->f2 = (double *)calloc(n, sizeof(double));
  h->g1 = (double *)calloc(n, sizeof(double));
  h->g2 = (double *)calloc(n, sizeof(double));
  h->psi = (double *)calloc((size_t)h->N, sizeof(double));
  return h;
}

/* first fluid neighbour of node n along -x, +x, -y, +y, -z, +z, or -1 */
static int64_t find_feeder(const lbo_params *p, const uint8_t *type, int64_t n) {
  static const int d[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
  int x = (int)(n % p->nx), y = (int)((n / p->nx) % p->ny), z = (int)(n / ((int64_t)p->nx * p->ny));
  for (int k = 0; k < 6; ++k) {
    if (p->nz == 1 && d[k][2] != 0) continue;
    int64_t m = nb(p, x, y, z, d[k][0], d[k][1], d[k][2]);
    if (type[m] == LBO_FLUID) return m;
  }
  return -1;
}

int lbo_set_geometry(lbo *h, const uint8_t *type, const double *rho1, const double *rho2,
                     const double *u) {
  const lbo_params *p = &h->p;
  if (p->walls_y || p->nci_mode != 0 || dr_on(p)) return -1;
  for (int64_t n = 0; n < h->N; ++n) {
    if (type[n] > LBO_OUTLET) return -1;
    if (type[n] == LBO_INLET || type[n] == LBO_OUTLET) {
      if (find_feeder(p, type, n) < 0) return -1;
      if (!(rho1[n] >= 0 && rho2[n] >= 0 && rho1[n] + rho2[n] > 0)) return -1;
    }
  }
  free(h->type); free(h->in1); free(h->in2); free(h->inu); free(h->feeder);
  h->type = (uint8_t *)malloc((size_t)h->N);
  memcpy(h->type, type, (size_t)h->N);
  h->in1 = (double *)calloc((size_t)h->N, sizeof(double));
  h->in2 = (double *)calloc((size_t)h->N, sizeof(double));
  h->inu = (double *)calloc(3 * (size_t)h->N, sizeof(double));
  h->feeder = (int64_t *)malloc(sizeof(int64_t) * (size_t)h->N);
  for (int64_t n = 0; n < h->N; ++n) {
    h->feeder[n] = -1;
    if (type[n] != LBO_INLET && type[n] != LBO_OUTLET) continue;
    h->feeder[n] = find_feeder(p, type, n);
    h->in1[n] = rho1[n];
    h->in2[n] = rho2[n];
    if (u && type[n] == LBO_INLET)
      for (int a = 0; a < h->dim; ++a) h->inu[a * h->N + n] = u[a * h->N + n];
  }
  return 0;
}

void lbo_destroy(lbo *h) {
  if (!h) return;
  free(h->f1); free(h->f2); free(h->g1); free(h->g2); free(h->psi);
  free(h->type); free(h->in1); free(h->in2); free(h->inu); free(h->feeder);
  free(h);
}

int64_t lbo_nodes(const lbo *h) { return h->N; }
int64_t lbo_time(const lbo *h) { return h->t; }

static int node_y(const lbo *h, int64_t n) { return (int)((n / h->p.nx) % h->p.ny); }

static int is_fluid(const lbo *h, int64_t n) {
  return h->type ? h->type[n] == LBO_FLUID : !is_wall_y(&h->p, node_y(h, n));
}

int lbo_init_fields(lbo *h, const double *rho1, const double *rho2, const double *u) {
  for (int64_t n = 0; n < h->N; ++n) {
    if (!is_fluid(h, n)) continue;
    if (!(rho1[n] >= 0) || !(rho2[n] >= 0) || !(rho1[n] + rho2[n] > 0)) return -1;
  }
  for (int64_t n = 0; n < h->N; ++n) {
    int wall = !is_fluid(h, n);
    double un[3] = {0, 0, 0};
    if (u)
      for (int a = 0; a < h->dim; ++a) un[a] = u[a * h->N + n];
    double w0 = h->w[0], al1, al2;
    for (int i = 0; i < h->Q; ++i)
      if (!h->c[i][0] && !h->c[i][1] && !h->c[i][2]) w0 = h->w[i];
    dr_alphas(&h->p, w0, &al1, &al2);
    for (int i = 0; i < h->Q; ++i) {
      if (dr_on(&h->p)) {
        h->f1[i * h->N + n] = wall ? 0.0 : equilibrium_k(al1, w0, h->w[i], h->c[i], rho1[n], un);
        h->f2[i * h->N + n] = wall ? 0.0 : equilibrium_k(al2, w0, h->w[i], h->c[i], rho2[n], un);
      } else {
        h->f1[i * h->N + n] = wall ? 0.0 : equilibrium_i(h->w[i], h->c[i], rho1[n], un);
        h->f2[i * h->N + n] = wall ? 0.0 : equilibrium_i(h->w[i], h->c[i], rho2[n], un);
      }
    }
  }
  h->t = 0;
  return 0;
}

void lbo_set_populations(lbo *h, const double *f1, const double *f2) {
  for (int64_t n = 0; n < h->N; ++n) {
    int wall = !is_fluid(h, n);
    for (int i = 0; i < h->Q; ++i) {
      h->f1[i * h->N + n] = wall ? 0.0 : f1[i * h->N + n];
      h->f2[i * h->N + n] = wall ? 0.0 : f2[i * h->N + n];
    }
  }
}

void lbo_get_populations(const lbo *h, double *f1, double *f2) {
  memcpy(f1, h->f1, sizeof(double) * (size_t)h->Q * (size_t)h->N);
  memcpy(f2, h->f2, sizeof(double) * (size_t)h->Q * (size_t)h->N);
}

/* steps 1-2: psi on fluid nodes, then wall rows copied from their neighbour */
static void compute_psi(lbo *h) {
  const lbo_params *p = &h->p;
#pragma omp parallel for schedule(static) if (h->N >= LBO_PAR_MIN)
  for (int64_t n = 0; n < h->N; ++n) {
    if (!is_fluid(h, n)) continue;
    double r1 = 0, r2 = 0;
    for (int i = 0; i < h->Q; ++i) {
      r1 += h->f1[i * h->N + n];
      r2 += h->f2[i * h->N + n];
    }
    h->psi[n] = dr_on(p) ? (r1 - p->rho_ratio * r2) / (r1 + p->rho_ratio * r2) : (r1 - r2) / (r1 + r2);
  }
  if (h->type) {
    /* inlets: their prescribed composition; outlets: their feeder's psi */
    for (int64_t n = 0; n < h->N; ++n) {
      if (h->type[n] == LBO_INLET) h->psi[n] = (h->in1[n] - h->in2[n]) / (h->in1[n] + h->in2[n]);
      else if (h->type[n] == LBO_OUTLET) h->psi[n] = h->psi[h->feeder[n]];
    }
    /* solids: w_i-weighted mean of the non-solid neighbours (0 without any) */
    for (int64_t n = 0; n < h->N; ++n) {
      if (h->type[n] != LBO_SOLID) continue;
      int x = (int)(n % p->nx), y = node_y(h, n), z = (int)(n / ((int64_t)p->nx * p->ny));
      double sw = 0, sp = 0;
      for (int i = 0; i < h->Q; ++i) {
        if (h->c[i][0] == 0 && h->c[i][1] == 0 && h->c[i][2] == 0) continue;
        int64_t m = nb(p, x, y, z, h->c[i][0], h->c[i][1], h->c[i][2]);
        if (h->type[m] == LBO_SOLID) continue;
        sw += h->w[i];
        sp += h->w[i] * h->psi[m];
      }
      h->psi[n] = sw > 0 ? sp / sw : 0.0;
    }
  }
  if (p->walls_y) {
    for (int z = 0; z < p->nz; ++z)
      for (int x = 0; x < p->nx; ++x) {
        int64_t b = x + (int64_t)p->nx * ((int64_t)p->ny * z);
        h->psi[b] = h->psi[b + p->nx];
        int64_t t = x + (int64_t)p->nx * ((p->ny - 1) + (int64_t)p->ny * z);
        h->psi[t] = h->psi[t - p->nx];
      }
  }
}

/* total force at a fluid node of the current state (psi already computed) */
static void node_force(lbo *h, int x, int y, int z, double G[3], double F[3], int32_t *hit,
                       double Frep[3], double *margin) {
  node_nci(&h->p, h->Q, h->c, h->w, h->psi, h->type, x, y, z, G, hit, Frep, margin);
  for (int a = 0; a < 3; ++a) F[a] = h->p.force[a] + Frep[a];
  if (h->dim == 2) F[2] = 0.0;
}

static void step_once(lbo *h) {
  const lbo_params *p = &h->p;
  const int Q = h->Q;
  const int64_t N = h->N;
  compute_psi(h);
  /* steps 3-8: collision at every fluid node into g1/g2 */
#pragma omp parallel for schedule(static) if (h->N >= LBO_PAR_MIN)
  for (int64_t n = 0; n < N; ++n) {
    int x = (int)(n % p->nx), y = (int)((n / p->nx) % p->ny), z = (int)(n / ((int64_t)p->nx * p->ny));
    if (!is_fluid(h, n)) continue;
    double G[3], F[3], Frep[3];
    int32_t hit;
    node_force(h, x, y, z, G, F, &hit, Frep, NULL);
    double a1[QMAX], a2[QMAX], o1[QMAX], o2[QMAX];
    for (int i = 0; i < Q; ++i) {
      a1[i] = h->f1[i * N + n];
      a2[i] = h->f2[i * N + n];
    }
    collide(p, Q, h->c, h->w, a1, a2, G, F, o1, o2);
    for (int i = 0; i < Q; ++i) {
      h->g1[i * N + n] = o1[i];
      h->g2[i * N + n] = o2[i];
    }
  }
  /* open boundaries: post-collision state of inlet and outlet nodes from
   * their feeders' post-collision populations */
  if (h->type) {
    for (int64_t n = 0; n < N; ++n) {
      if (h->type[n] != LBO_INLET && h->type[n] != LBO_OUTLET) continue;
      const int64_t f = h->feeder[n];
      double r1 = 0, r2 = 0, j[3] = {0, 0, 0};
      for (int i = 0; i < Q; ++i) {
        double a = h->g1[i * N + f], b = h->g2[i * N + f];
        r1 += a;
        r2 += b;
        for (int d = 0; d < 3; ++d) j[d] += h->c[i][d] * (a + b);
      }
      double rho = r1 + r2, e1, e2, ub[3];
      if (h->type[n] == LBO_INLET) {
        /* prescribed velocity and composition, the feeder's density */
        double fr = h->in1[n] / (h->in1[n] + h->in2[n]);
        e1 = rho * fr;
        e2 = rho - e1;
        for (int d = 0; d < 3; ++d) ub[d] = d < h->dim ? h->inu[d * N + n] : 0.0;
      } else {
        /* prescribed density, the feeder's velocity and composition */
        double ro = h->in1[n] + h->in2[n];
        e1 = ro * (r1 / rho);
        e2 = ro - e1;
        for (int d = 0; d < 3; ++d) ub[d] = j[d] / rho;
      }
      for (int i = 0; i < Q; ++i) {
        h->g1[i * N + n] = equilibrium_i(h->w[i], h->c[i], e1, ub);
        h->g2[i * N + n] = equilibrium_i(h->w[i], h->c[i], e2, ub);
      }
    }
  }
  /* step 9: pull streaming, half-way bounce-back from wall rows */
#pragma omp parallel for schedule(static) if (h->N >= LBO_PAR_MIN)
  for (int64_t n = 0; n < N; ++n) {
    int x = (int)(n % p->nx), y = (int)((n / p->nx) % p->ny), z = (int)(n / ((int64_t)p->nx * p->ny));
    if (!is_fluid(h, n)) continue;
    if (h->type) {
      for (int i = 0; i < Q; ++i) {
        int64_t src = nb(p, x, y, z, -h->c[i][0], -h->c[i][1], -h->c[i][2]);
        if (h->type[src] == LBO_SOLID) { /* half-way bounce-back */
          h->f1[i * N + n] = h->g1[h->opp[i] * N + n];
          h->f2[i * N + n] = h->g2[h->opp[i] * N + n];
        } else {
          h->f1[i * N + n] = h->g1[i * N + src];
          h->f2[i * N + n] = h->g2[i * N + src];
        }
      }
      continue;
    }
    for (int i = 0; i < Q; ++i) {
      int ys = y - h->c[i][1];
      if (p->walls_y && is_wall_y(p, ys)) {
        h->f1[i * N + n] = h->g1[h->opp[i] * N + n];
        h->f2[i * N + n] = h->g2[h->opp[i] * N + n];
      } else {
        int64_t src = nb(p, x, y, z, -h->c[i][0], -h->c[i][1], -h->c[i][2]);
        h->f1[i * N + n] = h->g1[i * N + src];
        h->f2[i * N + n] = h->g2[i * N + src];
      }
    }
  }
  h->t += 1;
}

void lbo_step(lbo *h, int64_t n) {
  for (int64_t s = 0; s < n; ++s) step_once(h);
}

/* moments and physical velocity u = (j + F/2)/rho at one node */
static void node_moments(lbo *h, int64_t n, double *r1, double *r2, double j[3]) {
  *r1 = *r2 = 0;
  j[0] = j[1] = j[2] = 0;
  for (int i = 0; i < h->Q; ++i) {
    double a = h->f1[i * h->N + n], b = h->f2[i * h->N + n];
    *r1 += a;
    *r2 += b;
    for (int d = 0; d < 3; ++d) j[d] += h->c[i][d] * (a + b);
  }
}

void lbo_fields(lbo *h, double *rho1, double *rho2, double *u) {
  const lbo_params *p = &h->p;
  compute_psi(h);
#pragma omp parallel for schedule(static) if (h->N >= LBO_PAR_MIN)
  for (int64_t n = 0; n < h->N; ++n) {
    int x = (int)(n % p->nx), y = (int)((n / p->nx) % p->ny), z = (int)(n / ((int64_t)p->nx * p->ny));
    if (!is_fluid(h, n)) {
      rho1[n] = rho2[n] = 0;
      for (int a = 0; a < h->dim; ++a) u[a * h->N + n] = 0;
      continue;
    }
    double r1, r2, j[3], G[3], F[3], Frep[3];
    int32_t hit;
    node_moments(h, n, &r1, &r2, j);
    node_force(h, x, y, z, G, F, &hit, Frep, NULL);
    rho1[n] = r1;
    rho2[n] = r2;
    for (int a = 0; a < h->dim; ++a) u[a * h->N + n] = (j[a] + 0.5 * F[a]) / (r1 + r2);
  }
}

void lbo_observables(lbo *h, double out[8]) {
  const lbo_params *p = &h->p;
  compute_psi(h);
  for (int k = 0; k < 8; ++k) out[k] = 0;
  for (int64_t n = 0; n < h->N; ++n) { /* fixed index order */
    int x = (int)(n % p->nx), y = (int)((n / p->nx) % p->ny), z = (int)(n / ((int64_t)p->nx * p->ny));
    if (!is_fluid(h, n)) continue;
    double r1, r2, j[3], G[3], F[3], Frep[3], uu = 0, ux;
    int32_t hit;
    node_moments(h, n, &r1, &r2, j);
    node_force(h, x, y, z, G, F, &hit, Frep, NULL);
    double rho = r1 + r2;
    out[0] += r1;
    out[1] += r2;
    for (int a = 0; a < 3; ++a) {
      double ph = j[a] + 0.5 * F[a];
      out[2 + a] += ph;
      uu += (ph / rho) * (ph / rho);
    }
    ux = (j[0] + 0.5 * F[0]) / rho;
    out[5] += ux;
    out[6] += r1 / rho * ux;
    if (sqrt(uu) > out[7]) out[7] = sqrt(uu);
  }
  out[5] /= p->nx;
  out[6] /= p->nx;
}

void lbo_diagnostics(lbo *h, double *psi, double *G, double *Frep, int32_t *hit, double *margin) {
  const lbo_params *p = &h->p;
  compute_psi(h);
  memcpy(psi, h->psi, sizeof(double) * (size_t)h->N);
#pragma omp parallel for schedule(static) if (h->N >= LBO_PAR_MIN)
  for (int64_t n = 0; n < h->N; ++n) {
    int x = (int)(n % p->nx), y = (int)((n / p->nx) % p->ny), z = (int)(n / ((int64_t)p->nx * p->ny));
    double g[3] = {0, 0, 0}, F[3], fr[3] = {0, 0, 0}, mg = INFINITY;
    int32_t ht = 0;
    if (is_fluid(h, n)) node_force(h, x, y, z, g, F, &ht, fr, &mg);
    for (int a = 0; a < 3; ++a) {
      G[a * h->N + n] = g[a];
      Frep[a * h->N + n] = fr[a];
    }
    hit[n] = ht;
    margin[n] = mg;
  }
}
