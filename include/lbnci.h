/*
 * lbnci.h -- C ABI of the MI355X colour-gradient lattice Boltzmann library
 * with near-contact interactions (NCI).
 *
 * The method is the one in the Materials and Methods section of Montessori,
 * Tiribocchi, Bonaccorso, Lauricella & Succi, "Lattice Boltzmann simulations
 * capture the multiscale physics of soft flowing crystals" (2019):
 *   Eq. (CGLBE)   two population sets f_i^k (k = 1 dispersed, 2 continuous)
 *                 streamed along c_i with dt = 1 on D3Q27 (D2Q9 in 2-D);
 *   moments       rho^k = sum_i f_i^k, rho u = sum_k sum_i c_i f_i^k;
 *   collision     Omega = Omega3[Omega1 + Omega2]: single-tau BGK relaxation
 *                 (mixture viscosity), perturbation (interfacial tension),
 *                 Latva-Kokko recolouring (segregation);
 *   Eq. (near_c)  F_rep = -A_h[h(x)] n delta_I, n = -grad psi/|grad psi|,
 *                 psi = (rho1-rho2)/(rho1+rho2), delta_I = |grad psi|/2,
 *                 A_h = A (h <= h_min), A (h_min/h)^3 (h <= h_max), 0 beyond;
 *   forcing       exact difference method, F = body force + F_rep.
 * The operator formulas the paper only names, wall treatment and tie rules
 * are fixed readings, documented with the project.
 *
 * Conventions
 *   - Node index n = x + nx*(y + ny*z), x fastest, for every array.
 *   - Host arrays are caller-owned; they are copied synchronously.
 *   - Device state is owned by the handle (hipMalloc at lb_create).
 *   - lb_step is asynchronous on the handle's HIP stream; lb_observables,
 *     lb_get_fields and lb_get_populations synchronise that stream.
 *   - Every call returns 0 (LB_OK) or a negative LB_E* code; the message of
 *     the last failure on the calling thread is lb_last_error().
 *   - Wall rows (walls_y = 1: y = 0 and y = ny-1) are solid.  Their entries in
 *     field/population arrays are ignored on input and 0 on output.
 */
#ifndef LBNCI_H
#define LBNCI_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_OK 0
#define LB_EINVAL (-1)   /* invalid argument or parameter                 */
#define LB_ENOMEM (-2)   /* device or host allocation failed              */
#define LB_EDEVICE (-3)  /* a HIP runtime call failed                     */
#define LB_ENUMERIC (-4) /* NaN/Inf detected in the observables            */
#define LB_ESTATE (-5)   /* call out of order (e.g. step before init)      */

typedef struct lb_handle lb_handle; /* opaque, owned by the library */

typedef enum { LB_D2Q9 = 0, LB_D3Q27 = 1 } lb_lattice;

/* Population storage (stored quantity: deviation s_i = f_i/w_i - 1 of the
 * post-collision total population from its lattice weight, plus per-node
 * colour scalars from which both components are rebuilt exactly):
 *   LB_STORE_FP32      s_i in FP32, colour fraction in FP64, FP64 arithmetic
 *   LB_STORE_FP16_DEV  s_i in FP16 (rest direction FP32, closing the node
 *                      mass exactly), FP32 arithmetic
 *   LB_STORE_BF16_DEV  as FP16_DEV with BF16
 *   LB_STORE_FP32_F32  s_i in FP32 with FP32 arithmetic throughout        */
typedef enum {
  LB_STORE_FP32 = 0,
  LB_STORE_FP16_DEV = 1,
  LB_STORE_BF16_DEV = 2,
  LB_STORE_FP32_F32 = 3
} lb_storage;

typedef struct {
  int32_t lattice;     /* lb_lattice                                           */
  int32_t nx, ny, nz;  /* lattice size; nz == 1 for D2Q9                       */
  int32_t walls_y;     /* 0: periodic in y; 1: half-way bounce-back walls at
                          y = 0 and y = ny-1 (x and z always periodic)         */
  double tau;          /* BGK relaxation time (> 1/2); nu = (tau - 1/2)/3      */
  double A_s;          /* perturbation amplitude; sigma = 2 A_s tau / 9        */
  double beta;         /* recolouring parameter, [0, 1]                        */
  double A_nci;        /* NCI strength A (>= 0; 0 switches NCI off)            */
  double h_min, h_max; /* NCI range in lattice spacings (paper: 2 and 4),
                          0 < h_min <= h_max <= 4                              */
  double force[3];     /* uniform body-force density (= -grad p)              */
  int32_t storage;     /* lb_storage                                           */
  int32_t obs_every;   /* record observables every k steps inside lb_step
                          (feeds the convergence test); 0 = only on request    */
  int32_t conv_window; /* convergence window W in recorded samples (0 = off)  */
  int32_t conv_m;      /* consecutive windows required                         */
  double conv_eps;     /* relative change of the windowed flow rate           */
  double tau2;         /* viscosity-ratio variant: relaxation time of
                          component 2 (> 1/2), tau then being component 1's;
                          a node relaxes at 1/tau_mix = (rho1/rho)/tau +
                          (rho2/rho)/tau2.  0 = one mixture tau (the paper's
                          model)                                              */
  int32_t nci_mode;    /* 0: the integer NCI probe (h = first s in
                          1..floor(h_max) with psi(x + round(s n)) >= psi(x),
                          marching stopped by walls; A_h of Eq. near_c).
                          1: continuous-NCI variant (not the paper's rule):
                          psi sampled at x + s n, s = 1..ceil(h_max), by
                          multilinear interpolation (rows clamped into the
                          fluid with walls), h at the linear crossing of the
                          last two samples (1 for s = 1), A_h shifted to
                          A ((h_min/h)^3 - q)/(1 - q), q = (h_min/h_max)^3, so
                          F_rep is continuous in the fields.  Other values
                          are LB_EINVAL.                                      */
  double rho_ratio;    /* density-ratio variant (an extension following the
                          colour-gradient model the paper builds on): gamma =
                          rho_1^0/rho_2^0 > 0; 0 = equal densities (the
                          paper's model).  Component k relaxes towards
                          E_i^k = rho_k phi_i^k + w_i rho_k (3 c.u + 4.5 (c.u)^2
                          - 1.5 u.u), phi_0^k = alpha_k, phi_i^k = (1 - alpha_k)
                          w_i/(1 - w_0), sound speed c_k^2 = (1 - alpha_k)/
                          (3 (1 - w_0)); recolouring weights the colour term by
                          (rho1 phi_i^1 + rho2 phi_i^2)/rho^2; psi =
                          (rho1 - gamma rho2)/(rho1 + gamma rho2).              */
  double alpha1;       /* rest fraction alpha_1 of component 1 (density-ratio
                          variant); alpha_2 = 1 - gamma (1 - alpha_1) so that
                          the reference densities have equal pressure.  Needs
                          0 < alpha_1 < 1 and 0 < alpha_2 < 1 (LB_EINVAL)     */
  double mass_tol;     /* mass-drift guard (>= 0; 0 = off): a recorded sample
                          (obs_every) whose component mass differs from that
                          of the first recorded sample after initialisation
                          by more than mass_tol times the total mass raises
                          flag bit 1 and makes lb_step / lb_observables return
                          LB_ENUMERIC.  Both components are conserved exactly
                          by the method (Eq. CGLBE streams and the collision
                          keeps each rho^k), so drift means lost precision.  */
} lb_params;

/* Observables of the current state, accumulated in FP64 in a fixed order:
 *   mass[k]  = sum_x rho^k
 *   mom      = sum_x (j + F/2)             (physical momentum, EDM)
 *   Q        = sum_x u_x / nx              (flow rate through a cross-section)
 *   Q_d      = sum_x (rho1/rho) u_x / nx   (dispersed-phase flow rate)
 *   umax     = max_x |u|,  u = (j + F/2)/rho
 *   converged: windowed-Q test satisfied (conv_window > 0)
 *   flags    : bit 0 NaN/Inf seen in any evaluated observable; bit 1 mass
 *              drift beyond mass_tol at a recorded sample (sticky until the
 *              next lb_init_fields / lb_set_populations)                 */
typedef struct {
  int64_t step;
  double mass[2];
  double mom[3];
  double Q, Q_d, umax;
  double Q_window;     /* mean Q over the last complete window (0 if none) */
  int32_t converged;
  int32_t flags;
} lb_obs;

/* Creates a lattice on the current HIP device with the model parameters of
 * Materials and Methods (lattice of Eq. CGLBE, relaxation time, perturbation
 * amplitude, recolouring parameter, NCI strength and range of Eq. near_c,
 * body force).  hip_stream: a hipStream_t (NULL = default stream) on which
 * all work of the handle is enqueued.  *out receives the handle, which the
 * caller releases with lb_destroy.
 * Errors: LB_EINVAL (tau <= 1/2, beta outside [0,1], sizes <= 0, nz != 1 with
 * D2Q9, walls with ny < 3, h_min > h_max, h_max > 4 or h_min <= 0, A_nci < 0,
 * unknown storage, more than 2^29 nodes), LB_ENOMEM, LB_EDEVICE.  Device
 * memory per node (two state copies plus psi and rho1): D3Q27 about 272 B
 * with FP32 storage and 152 B with FP16/BF16, so 2^29 nodes fit in 288 GB
 * (lb_init_fields / lb_set_populations hold 2 Q FP64 values per node more
 * until the first lb_step has consumed them). */
int lb_create(const lb_params *p, void *hip_stream, lb_handle **out);

/* Initial state of the two population sets of Eq. CGLBE,
 * f_i^k(x,0) = E_i(rho^k(x), u(x)) with the second-order equilibrium,
 * computed on the host in FP64.  rho1, rho2: N doubles each;
 * u: dim*N doubles (u_x block, u_y block[, u_z block]) or NULL for rest.
 * Errors: LB_EINVAL on negative/NaN densities or rho1+rho2 <= 0 at a fluid
 * node.  Resets the step counter and the convergence state. */
int lb_init_fields(lb_handle *h, const double *rho1, const double *rho2, const double *u);

/* Arbitrary initial state of the two population sets of Eq. CGLBE: f1, f2
 * hold Q*N doubles each in layout [i][n] with the direction order of
 * lb_lattice_tables (caller-owned, copied).  Errors as lb_init_fields, and
 * LB_EINVAL on a non-finite population. */
int lb_set_populations(lb_handle *h, const double *f1, const double *f2);

/* Advance n >= 0 steps of Eq. CGLBE (collide, then pull-stream; one step is
 * the whole update of Materials and Methods: densities and psi, colour
 * gradient, NCI force of Eq. near_c, BGK + perturbation + recolouring with
 * exact-difference forcing, streaming).  Asynchronous on the handle's stream.
 * Errors: LB_EINVAL (n < 0), LB_ESTATE before initialisation, LB_EDEVICE on
 * launch failure, LB_ENUMERIC when a step recorded before this call (obs_every
 * > 0) saw a NaN/Inf or a mass drift beyond mass_tol: the flags of recorded
 * steps reach the host asynchronously, so a failure shows at the next
 * lb_step after the stream has passed the recording, and always at
 * lb_observables.  The steps of the failing call are not run. */
int lb_step(lb_handle *h, int64_t n);
/* Captures and instantiates, ahead of the first lb_step, the replay graphs
 * lb_step uses for windows of plain steps (both ping-pong copies); optional,
 * lb_step otherwise builds them on first use.  Runs no step and changes no
 * state.  Returns LB_OK, or LB_EDEVICE if capture failed (lb_step then uses
 * plain launches; its results are identical either way). */
int lb_prepare(lb_handle *h);
/* Measurement support: lb_step(h, n) bracketed by two HIP events recorded on
 * the handle's stream; *ms receives the device time between them.
 * Synchronises the stream.  Errors as lb_step; LB_EINVAL for a NULL ms. */
int lb_step_timed(lb_handle *h, int64_t n, double *ms);
/* 1 while lb_step replays windows of 16 plain steps (no observable recording
 * inside, profiling off) from a captured hipGraph, 0 after a capture failed
 * (plain launches from then on; the results are identical either way). */
int lb_graphs(const lb_handle *h);

/* Observables of the current state (synchronises the stream): component
 * masses and momentum (moments paragraph of Materials and Methods), flow
 * rate Q and dispersed flow rate Q_d (the paper's observable, Results /
 * Fig. 3), umax, and the windowed convergence state.
 * Returns LB_ENUMERIC if a NaN/Inf or a mass drift was flagged (out is still
 * filled). */
int lb_observables(lb_handle *h, lb_obs *out);

/* Current fields: the component densities rho1, rho2 (N doubles each) and
 * the physical velocity of the exact difference method u = (j + F/2)/rho
 * (dim*N doubles), F the force of the next collision.  Host arrays,
 * caller-owned; synchronises the stream.  LB_ESTATE before initialisation. */
int lb_get_fields(lb_handle *h, double *rho1, double *rho2, double *u);

/* Allocation-free variant of lb_get_fields, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same outputs, bit for bit, as lb_get_fields; the
 * device staging of the FP64 fields goes through a fixed array of
 * LB_STATIC_SCRATCH_BYTES that each GPU the library runs on holds for the
 * life of the process, so no hipMalloc/hipFree or allocating library call is
 * made.  Limit: (2 + dim) * N doubles must fit, i.e. N <= 2^21 nodes in 2-D
 * and N <= 1,677,721 in 3-D (larger lattices: LB_EINVAL, nothing run).  The
 * handle's device must be current (LB_EINVAL otherwise).  Every call on one
 * GPU shares that GPU's array and leaves its contents behind; calls that
 * overlap on one GPU (other threads, or handles on other streams) race and
 * must be serialised by the caller.  Synchronises the handle's stream.
 * Errors: LB_EINVAL, LB_ESTATE before initialisation, LB_EDEVICE. */
#define LB_STATIC_SCRATCH_BYTES (64u << 20)
int lb_get_fields_static(lb_handle *h, double *rho1, double *rho2, double *u);

/* Current post-streaming populations of Eq. CGLBE, f1, f2 ([i][n], Q*N
 * doubles each, caller-owned host arrays), rebuilt from the stored state;
 * synchronises the stream. */
int lb_get_populations(lb_handle *h, double *f1, double *f2);

/* Per-node diagnostics of the current state: psi (N doubles; wall rows hold
 * the copied value), the near-contact force F_rep of Eq. near_c (dim*N
 * doubles) and the probe's hit distance h (N int32, 0 = no hit).  Any
 * pointer may be NULL; synchronises the stream. */
int lb_get_nci(lb_handle *h, double *psi, double *frep, int32_t *hit);

/* Releases the handle and its device memory (waits for its stream first);
 * NULL is ignored. */
void lb_destroy(lb_handle *h);

/* Lattice tables (D2Q9, or the D3Q27 lattice of Materials and Methods) in the
 * library's direction order: c[Q*3] (x,y,z), w[Q]; either pointer may be
 * NULL.  Returns Q, or LB_EINVAL for an unknown lattice. */
int lb_lattice_tables(int32_t lattice, int32_t *c, double *w);

/* Step counter of the handle (number of completed lb_step steps). */
int64_t lb_time(const lb_handle *h);

/* Device bytes held by the handle (state, phase field, scratch). */
int64_t lb_device_bytes(const lb_handle *h);

/* Per-kernel timing with HIP events recorded on the handle's stream around
 * every k_phase and k_main launch of lb_step (measurement support; adds one
 * event per launch).  lb_kernel_times synchronises the stream, returns the
 * summed durations (ms) and launch count since the last call, and resets. */
int lb_profile(lb_handle *h, int enable);
int lb_kernel_times(lb_handle *h, double *ms_phase, double *ms_main, int64_t *launches);

/* A HIP stream for lb_create / lb_batch_create / lb_copy_probe: non-blocking
 * (no implicit wait on the default stream), default priority, on the current
 * device of the HIP runtime this library is linked against.  Handles on
 * different streams run side by side (their kernels share the device); a
 * stream created by another copy of the HIP runtime in the same process (one
 * bundled with a Python framework, say) is not valid here.  *stream receives
 * the hipStream_t.  lb_stream_destroy waits for the stream's work, then
 * releases it; destroy every handle that uses the stream first.  Errors:
 * LB_EINVAL for a NULL pointer, LB_EDEVICE from the runtime. */
int lb_stream_create(void **stream);
int lb_stream_destroy(void *stream);

/* Achievable-bandwidth reference: a plain streaming copy of `bytes` bytes
 * (16-byte vector loads/stores) repeated `iters` times on the current device;
 * returns the average per-copy duration (ms) and the read+write rate (GB/s).
 * Allocates and frees two device buffers. */
int lb_copy_probe(int64_t bytes, int iters, void *hip_stream, double *ms, double *gbps);

/* ---- Node-type geometry (Results: droplet generation in a flow-focuser,
 * Fig. 1 -- a device with inlet channels, a striction and an outlet) --------
 * lb_set_geometry turns the periodic lattice into a device: type[n] is one of
 *   LB_NODE_FLUID  updated by the LB step;
 *   LB_NODE_SOLID  half-way bounce-back for its fluid neighbours; its psi
 *                  (for the colour gradient) is the w_i-weighted mean of the
 *                  psi of its non-solid neighbours (neutral wetting), 0 if
 *                  it has none; the NCI probe stops at it;
 *   LB_NODE_INLET  velocity inlet: after every collision it holds the
 *                  equilibrium at velocity u[n] and composition
 *                  rho1[n]/(rho1[n] + rho2[n]) with the density of its
 *                  feeder; psi = its composition;
 *   LB_NODE_OUTLET pressure outlet: the equilibrium at density
 *                  rho1[n] + rho2[n] with the velocity and composition of
 *                  its feeder; psi = the feeder's.
 * The feeder of an inlet/outlet node is its first fluid neighbour along -x,
 * +x, -y, +y, -z, +z (one is required).  The NCI probe also stops at inlet and
 * outlet nodes.  type, rho1, rho2 (N) and u (dim*N, may be NULL: zero inlet
 * velocity) are host arrays read during the call.  Requires walls_y == 0
 * (walls are solid nodes), nci_mode == 0 and rho_ratio == 0; call before lb_init_fields /
 * lb_set_populations (which then initialise fluid nodes only), once per
 * handle.  Errors: LB_EINVAL (bad type value, an inlet/outlet without a fluid
 * axis neighbour, invalid prescribed densities, walls_y or nci_mode set, an
 * extent not above h_max while A_nci > 0, a second call), LB_ENOMEM,
 * LB_EDEVICE.  Single lattices only (not batches). */
#define LB_NODE_FLUID 0
#define LB_NODE_SOLID 1
#define LB_NODE_INLET 2
#define LB_NODE_OUTLET 3
int lb_set_geometry(lb_handle *h, const uint8_t *type, const double *rho1, const double *rho2,
                    const double *u);

/* ---- Droplet-level analysis (Results: droplet count and volume, the
 * hex-n arrangements named by their number of droplet rows, vorticity of the
 * flow) ----------------------------------------------------------------
 * Droplets are the connected components of the dispersed phase: the fluid
 * nodes with psi = (rho1 - rho2)/(rho1 + rho2) > 0 in the current fields (the
 * rho1, rho2 of lb_get_fields, psi evaluated in FP64), under face adjacency
 * (4 neighbours in 2-D, 6 in 3-D), periodic in x and z, and in y when
 * walls_y == 0.  The label of a droplet is the smallest node index
 * n = x + nx*(y + ny*z) in it.  Both calls run one lattice pass in FIELDS mode
 * into a device arena that the handle allocates on first use (about 120 bytes
 * per node) and keeps until lb_destroy.  Lattices of 2^31 nodes or more are
 * rejected (LB_EINVAL).  LB_ESTATE before initialisation, LB_ENOMEM when the
 * arena cannot be allocated, LB_EDEVICE on a HIP failure. */
typedef struct {
  int64_t count;     /* number of droplets */
  int64_t dispersed; /* number of nodes with psi > 0 */
  int32_t rows;      /* droplet rows across the channel (hex-n): droplets of at least a
                        quarter of the mean volume, sorted by centroid y; a gap in y above
                        half the equivalent diameter (disk in 2-D, sphere in 3-D) of their
                        median volume starts a new row; 0 without droplets */
} lb_droplet_stats;

/* Labels the droplets of the current state and lists them in ascending label
 * order.  All outputs are host arrays owned by the caller; any may be NULL.
 *   label    N int32: each node's droplet label, -1 outside the dispersed phase;
 *   root     cap int64: the label of each listed droplet;
 *   volume   cap int64: its node count V_d;
 *   centroid 3*cap doubles, (x, y, z) per droplet: the root's coordinates plus
 *            the mean offset of the droplet's nodes from the root, each offset
 *            taken along periodic axes as the image in
 *            [-floor(L/2), L-1-floor(L/2)], the result moved back into [0, L)
 *            (meaningful for droplets shorter than half of each period).
 * Only the first min(count, cap) droplets are listed; stats->count is the
 * full count.  cap < 0 is LB_EINVAL.  Synchronises the stream. */
int lb_droplets(lb_handle *h, lb_droplet_stats *stats, int32_t *label, int64_t cap, int64_t *root,
                int64_t *volume, double *centroid);

/* Vorticity omega = curl u of the current velocity (the u of lb_get_fields)
 * by central differences between nearest nodes, (u(x+e) - u(x-e))/2 per
 * axis, wrapping along periodic axes; wall rows hold u = 0 and receive
 * omega = 0.  omega: host, N doubles for D2Q9 (omega_z), 3*N for D3Q27
 * (omega_x, omega_y, omega_z blocks).  Synchronises the stream. */
int lb_vorticity(lb_handle *h, double *omega);

/* Device time (ms) of the last lb_droplets and lb_vorticity calls: the FIELDS
 * pass plus the analysis kernels, between events on the handle's stream
 * (0 if the call has not been made).  Either pointer may be NULL. */
int lb_analysis_times(const lb_handle *h, double *ms_droplets, double *ms_vorticity);

/* ---- Batched stepping of many independent lattices ("channels") --------
 * For sweeps of the kind the paper runs over pressure gradient and NCI
 * strength (Results: flow rate versus driving), many small lattices of
 * uneven size are stepped together on one GPU.  All channels of a batch share
 * lattice type, storage and obs_every; sizes and physical parameters differ.
 * Channels with conv_window > 0 retire (stop stepping) once their windowed
 * flow-rate test is satisfied. */
typedef struct lb_batch lb_batch;
#define LB_BATCH_LAUNCH 0     /* per step: phase, main and bookkeeping launches over a
                                 tile table of all channels, replayed from a hipGraph */
#define LB_BATCH_PERSISTENT 1 /* one cooperative persistent launch for all steps; each
                                 channel synchronises only its own group of blocks */
#define LB_BATCH_AUTO 2       /* the configuration chosen by lb_batch_tune / set_config */

/* p: n parameter sets.  Creates n handles on the stream plus the tile tables
 * and persistent-launch groups.  Errors as lb_create, and LB_EINVAL when the
 * channels differ in lattice/storage/obs_every or ask for the continuous-NCI
 * variant (nci_mode 1 runs on single lattices only). */
int lb_batch_create(const lb_params *p, int32_t n, void *hip_stream, lb_batch **out);
/* As lb_init_fields for channel c (0 <= c < n). */
int lb_batch_init_fields(lb_batch *b, int32_t c, const double *rho1, const double *rho2,
                         const double *u);
/* Advances every active channel by n steps (synchronises the stream at the
 * end).  The first call after initialisation performs the explicit first step
 * of every channel as one plain step (channels must be initialised together).
 * Errors: LB_ESTATE (uninitialised channel), LB_EDEVICE (launch failure or a
 * channel barrier that did not complete within its spin limit). */
int lb_batch_step(lb_batch *b, int64_t n, int32_t mode);
/* Flags of every channel (n int32, the lb_obs flags bits) after the last
 * lb_batch_step, which returns LB_ENUMERIC when any channel has one set (the
 * other channels have still taken their steps). */
int lb_batch_flags(lb_batch *b, int32_t *flags);
int lb_batch_observables(lb_batch *b, int32_t c, lb_obs *out);
int lb_batch_get_fields(lb_batch *b, int32_t c, double *rho1, double *rho2, double *u);
/* Steps completed by channel c, whether it is still active, and the number of
 * blocks of its persistent group. */
int lb_batch_info(lb_batch *b, int32_t c, int64_t *steps, int32_t *active, int32_t *blocks);
/* 1 while both modes run from hipGraphs, 0 after a graph path failed and
 * direct launches are used. */
int lb_batch_graphs(lb_batch *b);
/* Autotuner: times each candidate configuration (execution mode; tile order:
 * 0 = each XCD receives a contiguous range of tiles, 1 = channel order; main
 * tile height 4/8/16 rows for D2Q9) over trial_steps real steps (they advance
 * the channels, plus 2 warm-up steps per candidate) and keeps the fastest as
 * the batch's configuration (used by mode LB_BATCH_AUTO).  best_ms_per_step
 * may be NULL. */
int lb_batch_tune(lb_batch *b, int32_t trial_steps, double *best_ms_per_step);
int lb_batch_set_config(lb_batch *b, int32_t mode, int32_t tile_order, int32_t main_by);
int lb_batch_get_config(lb_batch *b, int32_t *mode, int32_t *tile_order, int32_t *main_by);
void lb_batch_destroy(lb_batch *b);

/* Thread-local message of the last failure ("" if none). */
const char *lb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
