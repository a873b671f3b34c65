/*
 * lbo.h -- FP64 CPU oracle for the two-component colour-gradient lattice
 * Boltzmann method with near-contact interactions (NCI).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain reference that the GPU
 * library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no source with the GPU library.
 *
 * Method (Materials and Methods of Montessori, Tiribocchi, Bonaccorso,
 * Lauricella & Succi, "Lattice Boltzmann simulations capture the multiscale
 * physics of soft flowing crystals", 2019):
 *   - Eq. (CGLBE): two population sets f_i^k, k = 1 (dispersed), 2 (continuous),
 *     streamed along c_i with dt = 1; D3Q27 lattice (D2Q9 for 2-D boxes).
 *   - densities rho^k = sum_i f_i^k, momentum rho u = sum_k sum_i c_i f_i^k.
 *   - collision Omega = Omega3[Omega1 + Omega2]: BGK relaxation, Gunstensen-type
 *     perturbation (interfacial tension), Latva-Kokko recolouring.
 *   - order parameter psi = (rho1-rho2)/(rho1+rho2), normal n = -grad psi/|grad psi|.
 *   - Eq. (near_c): F_rep = -A_h[h(x)] n delta_I, delta_I = |grad psi|/2, with a
 *     second-order isotropic gradient; A_h = A for h <= h_min, ~h^-3 up to h_max,
 *     0 beyond.
 *   - forcing by the exact difference method.
 * Operator formulas that the paper only names are fixed by the readings listed
 * in DESIGN.md ("Readings of the paper").
 *
 * Parity pins: every function is pinned by tests in tests/test_oracle_*.py
 * against closed forms, hand-tabulated values and invariants.
 */
#ifndef LBO_H
#define LBO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { LBO_D2Q9 = 0, LBO_D3Q27 = 1 };
enum { LBO_FLUID = 0, LBO_SOLID = 1, LBO_INLET = 2, LBO_OUTLET = 3 };

typedef struct {
  int32_t lattice;          /* LBO_D2Q9 or LBO_D3Q27                         */
  int32_t nx, ny, nz;       /* nz == 1 for D2Q9; node index x + nx*(y + ny*z) */
  int32_t walls_y;          /* 1: rows y=0 and y=ny-1 are solid (bounce-back) */
  double tau;               /* BGK relaxation time (mixture)                  */
  double A_s;               /* perturbation amplitude                         */
  double beta;              /* recolouring parameter                          */
  double A_nci, h_min, h_max; /* NCI strength and range                       */
  double force[3];          /* uniform body-force density (= -grad p)         */
  double tau2;              /* relaxation time of component 2; 0: both use tau.
                               Otherwise tau is component 1's and the node's
                               1/tau_mix = (rho1/rho)/tau + (rho2/rho)/tau2  */
  int32_t nci_mode;         /* 0: R-NCI (integer march, nearest-node samples,
                               A_h of Eq. near_c); 1: continuous-NCI variant
                               (interpolated samples, continuous h, A_h shifted
                               to reach 0 at h_max)                          */
  double rho_ratio;         /* density-ratio variant: gamma = rho_1^0/rho_2^0
                               (> 0; 0 = equal densities, the paper's model) */
  double alpha1;            /* rest fraction of component 1's equilibrium;
                               alpha_2 = 1 - gamma (1 - alpha_1)             */
} lbo_params;

typedef struct lbo lbo;

/* lattice tables: c[Q*3] (x,y,z), w[Q], opp[Q].  Returns Q. */
int lbo_lattice(int lattice, int32_t *c, double *w, int32_t *opp);

lbo *lbo_create(const lbo_params *p);
void lbo_destroy(lbo *h);
int64_t lbo_nodes(const lbo *h);

/* Node types (N bytes, LBO_*) on the periodic lattice; requires walls_y = 0
 * and nci_mode = 0 and equal densities.  Every inlet/outlet needs a fluid neighbour along an axis
 * (its feeder).  Inlets take their composition rho1/(rho1+rho2) and velocity
 * u (dim*N, may be NULL) at their index, outlets their density rho1 + rho2.
 * Call before init_fields.  Returns 0, or -1 on an invalid mask. */
int lbo_set_geometry(lbo *h, const uint8_t *type, const double *rho1, const double *rho2,
                     const double *u);

/* f_i^k(x,0) = E_i(rho^k(x), u(x)); u may be NULL (u = 0).  u layout: dim
 * component-major blocks of N.  Returns 0 or -1 on invalid densities. */
int lbo_init_fields(lbo *h, const double *rho1, const double *rho2, const double *u);
/* Populations in layout [i][node] (Q blocks of N).  Wall-node entries ignored
 * on set and returned as 0 on get. */
void lbo_set_populations(lbo *h, const double *f1, const double *f2);
void lbo_get_populations(const lbo *h, double *f1, double *f2);

/* advance n steps (collide then pull-stream) */
void lbo_step(lbo *h, int64_t n);
int64_t lbo_time(const lbo *h);

/* fields at the current time: rho^k and the physical velocity
 * u = (j + F/2)/rho, F the force of the next collision.  Wall nodes -> 0. */
void lbo_fields(lbo *h, double *rho1, double *rho2, double *u);

/* observables at the current time, in fixed index order:
 * out[0..1] = mass of component 1, 2; out[2..4] = sum (j + F/2);
 * out[5] = Q = sum u_x / nx; out[6] = Q_d = sum (rho1/rho) u_x / nx;
 * out[7] = max |u|. */
void lbo_observables(lbo *h, double out[8]);

/* per-node diagnostics at the current time: psi (N, walls carry the copied
 * value), G (3N), F_rep (3N), hit distance h (N, 0 = none), and the decision
 * margin (N): the smallest of |G| (the probe's existence and direction are
 * ill-conditioned as |G| -> 0), |psi(y_s) - psi(x)| over probed sites and the
 * distance of a probed s*n component to a rounding tie; infinity when NCI is
 * off. */
void lbo_diagnostics(lbo *h, double *psi, double *G, double *Frep, int32_t *hit,
                     double *margin);

/* --- single-node operators, for unit pins ------------------------------- */
void lbo_equilibrium(int lattice, double rho, const double u[3], double *feq);
/* density-ratio variant: component equilibrium with rest fraction alpha */
void lbo_equilibrium_k(int lattice, double alpha, double rho, const double u[3], double *feq);
/* one collision at a node: inputs f1,f2 (Q each), gradient G and total force F;
 * outputs the post-recolouring populations. */
void lbo_collide_node(const lbo_params *p, const double *f1, const double *f2,
                      const double G[3], const double F[3], double *out1, double *out2);
double lbo_A_h(double h, double A, double h_min, double h_max);
/* continuous-NCI variant: A for h <= h_min, A ((h_min/h)^3 - q)/(1 - q) with
 * q = (h_min/h_max)^3 up to h_max, 0 beyond (continuous at both ends) */
double lbo_A_h_shifted(double h, double A, double h_min, double h_max);
/* gradient and NCI at one node of a given psi field (N values, wall rows
 * already holding their copied values). */
void lbo_node_nci(const lbo_params *p, const double *psi, int64_t node, double G[3],
                  int32_t *hit, double Frep[3]);

#ifdef __cplusplus
}
#endif
#endif
