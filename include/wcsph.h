/*
 * wcsph.h -- C ABI of the MI355X planar WCSPH hot path (libwcsph.so).
 *
 * The library advances the per-step particle pipeline of a planar
 * weakly-compressible SPH model of hydrodynamic ram (a rigid disk driven
 * through a water channel): cell-linked-list neighbour search, Wendland C2
 * continuity (with delta diffusion) and momentum sums, Tait EOS with a
 * cavitation cutoff, Monaghan artificial viscosity, Adami ghost particles on
 * the channel walls and the moving disk, and a predictor-corrector update.
 * Section / equation names below refer to the paper "Verification,
 * Sensitivity, and Operating Limits of a GPU-Accelerated Planar WCSPH Model
 * for Hydrodynamic Ram".
 *
 * Conventions
 *  - SI units. The fluid box is [0,L]x[0,W]; the disk moves along +x.
 *  - Every function returns wcsph_status; nothing throws across the ABI.
 *  - Host pointers are caller-owned and only read/written during the call.
 *    Device memory is owned by the context; it is obtained through the
 *    caller's allocator (or hipMalloc when none is given) at create time.
 *  - Work is queued on the stream given at create (it must not be the
 *    legacy NULL stream: the step is captured into a HIP graph on it).
 *    wcsph_step returns without waiting; every read_* / get_* / export_*
 *    call synchronises the stream first.
 *  - A context is not thread-safe; use one context per host thread.
 *  - On error the context keeps its previous state when possible and
 *    wcsph_last_error() describes the failure. After WCSPH_E_HIP the
 *    context must only be destroyed.
 */
#ifndef WCSPH_H
#define WCSPH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WCSPH_OK = 0,
  WCSPH_E_INVALID = 1,  /* bad argument or parameter; nothing was changed */
  WCSPH_E_OOM = 2,      /* an allocation failed; the context is still destroyable */
  WCSPH_E_HIP = 3,      /* a HIP runtime call failed */
  WCSPH_E_STATE = 4,    /* call not valid in the current state (NULL / destroyed ctx) */
  WCSPH_E_UNSTABLE = 5, /* a diagnostic found a non-finite value or an escaped particle,
                           or a cell held more particles than a cell bucket takes (64) */
  WCSPH_E_RANGE = 6     /* a size argument is too small for the data */
} wcsph_status;

#define WCSPH_MAX_PROBES 16

typedef struct wcsph_ctx wcsph_ctx;

/* Optional device allocator (e.g. a framework's caching allocator).
 * alloc returns device memory of at least `bytes` bytes or NULL; free
 * releases it. `stream` is the context's stream. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* stream, void* user);
  void* user;
} wcsph_allocator;

/* Problem and scheme parameters (copied at create).
 *  kernel     : kernel_type 0 = Wendland C2 (the hot path's), 1 = the cubic
 *               B-spline of eq. cubic-kernel (the paper's); support 2h both.
 *  geometry   : channel [0,L]x[0,W], lattice spacing dx, h = h_over_dx dx
 *               (1.3: SPH Fundamentals), cell edge cell_size >= 2h (<= 0 -> the
 *               smallest float >= 2h), ghost_layers wall-ghost lattice rows.
 *  material   : rho0, Tait c0 and gamma (B = rho0 c0^2 / gamma), cavitation
 *               cutoff p_cav (< 0, eq. eos text). eos_type 0 = Tait; 1 = the
 *               Mie-Grueneisen law of eq. eos with the specific internal
 *               energy held at zero (no energy equation is evolved, so its
 *               (gamma0 + a mu) rho e term vanishes): with mu = rho/rho0 - 1
 *               capped at mg_mu_max and C = c0, p = rho0 C^2 mu [1 +
 *               (1 - mg_gamma0/2) mu] / [1 - (mg_s1 - 1) mu]^2 in compression,
 *               rho0 C^2 mu in tension, the same cutoff, c^2 = dp/drho; then
 *               ghost_rho_mode 1 is its inverse, e_el its elastic energy, and
 *               gamma is unused. Requires mg_s1 >= 1, 0 <= mg_gamma0 < 2,
 *               mg_mu_max > 0, (mg_s1 - 1) mg_mu_max < 0.9. Batched
 *               instances may mix the two laws. The reverse sweep takes Tait
 *               only.
 *  scheme     : Monaghan alpha and eta2 (eq. artificial-viscosity), beta of
 *               the quadratic term beta mu^2 / rho_bar that the paper omits
 *               (0 = linear term only, the paper's form), delta
 *               diffusion coefficient, eps_xsph (eq. xsph), dynamic viscosity
 *               mu_dyn (laminar term), CFL number (eq. cfl), gravity_y,
 *               density band [rho_lo, rho_hi] rho0 (Density Summation),
 *               wall pull-back eps_wall (Channel Walls).
 *  disk       : radius disk_R (0 -> no disk) starting at (disk_x0, disk_y0),
 *               n_disk_ghosts ring ghosts of mass rho0 dx 2 pi R / N_g
 *               (eq. adami-p text), ghost_rho_mode 0 = linear acoustic branch
 *               rho0 (1 + p / (rho0 c0^2)) (eq. adami-v), 1 = Tait inverse,
 *               disk_mass (per unit depth, kg/m) for the disk kinetic energy
 *               diagnostic and the coupled disk's inertia.
 *  kinematics : kin_mode 0 = ramp (eq. velocity-ramp) over kin_t_ramp to kin_v0
 *               then constant deceleration kin_coef (m/s^2); 1 = ramp then
 *               quadratic drag dv/dt = -kin_coef v^2 (eq. drag); 2 = two-way
 *               coupling (the extension named with the energy audit and in
 *               the Conclusions): the ramp, then from the first step starting
 *               at t >= kin_t_ramp the disk obeys disk_mass dv/dt = -f, f the
 *               x force of the ring on the fluid at the step midpoint (the
 *               FP64 sum of the per-ghost forces), trapezoidal position; the
 *               boundary work then uses the step's mean disk velocity, so that
 *               e_disk + w_boundary stays constant. kin_coef is unused;
 *               disk_mass > 0 is required. 3 = a tabulated prescribed
 *               motion (rows set with wcsph_set_disk_kinematics mode 3).
 *  probes     : n_probes points (x, y) where the Shepard-averaged fluid
 *               pressure is recorded every step.
 *  output     : diag_every steps between diagnostic records; init_mode 0 =
 *               fluid at rest at rho0, 1 = hydrostatic density; audit 1 =
 *               record the energy audit terms (single-instance contexts; the
 *               second pair pass then carries four more sums per pair).
 *  update     : scheme 0 = continuity with the delta term and the
 *               predictor-corrector (two evaluations per step); 1 = the
 *               paper's scheme as published, one evaluation per step:
 *               density by summation (eq. density-sum) over the fluid and
 *               ghosts in support, the particle itself included, with masses
 *               normalised so that the undisturbed square lattice sums to
 *               rho0 (fluid and wall ghosts rho0 / sum_j W_j, the ring that
 *               mass per dx of arc), clamped to [rho_lo, rho_hi] rho0 (Density
 *               Summation); delta unused; the leapfrog of Time Integration
 *               with a merged kick v^(n+1/2) = v^(n-1/2) + (dt^(n-1) + dt^n)/2
 *               a^n (dt^(-1) = 0 after create, set_fluid and load), drift
 *               r^(n+1) = r^n + dt^n (v^(n+1/2) + the XSPH correction), and a
 *               specific internal energy e^(n+1) = e^n + dt^n de/dt, de/dt =
 *               (1/2) sum_j m_j Pi_ij v_ij . grad W_ij (the artificial
 *               viscosity's heating, over fluid and ghosts); with eos_type 1
 *               the Mie-Grueneisen law gains its energy term (mg_gamma0 +
 *               mg_a mu) rho e (mg_gamma0 rho e in tension), rho = rho0 (1 +
 *               mu) at the capped mu; c stays the e = 0 law's. The stored
 *               state is then (r^(n+1), v^(n+1/2), e^(n+1)) with rho the
 *               step's summed density (at r^n), which is what the readers,
 *               the diagnostics (ke of v^(n+1/2), e_el of that rho, e_th = sum
 *               m e) and save/load see. Scheme 1 requires kin_mode != 2 and
 *               audit = 0, and every instance of a batch must share it; the
 *               reverse sweep takes scheme 0 only.
 *  axisym     : 1 = the axisymmetric r-z form, the extension the Conclusions
 *               rank first (it restores the out-of-plane relief the planar
 *               section discards, Formulation Comparison): the plane is the
 *               meridian half-plane through the tank axis, x the axial
 *               coordinate and y the radius, so [0,L]x[0,W] is a tank of
 *               radius W with its axis on y = 0, and the disk is a sphere
 *               whose centre must lie on the axis (disk_y0 = 0). Each fluid
 *               particle is a ring of fixed mass M = 2 pi r0 rho0 dx^2 (r0 its
 *               radius at set-up; wcsph_set_fluid keeps these masses) and
 *               enters the pair sums with the planar mass M / (2 pi max(r,
 *               dx/2)); the continuity equation adds the hoop part of the
 *               divergence, -rho v_r / max(r, dx/2); the wall-ghost layers
 *               below the axis mirror the fluid (the Adami pressure, axial
 *               velocity kept, radial reversed) and are switched off inside
 *               the sphere. mass, mom, ke, e_el and w_boundary (with the
 *               ring's force on the fluid and, for kin_mode 2, the sphere's
 *               motion) are then 3D values: each particle weighs its ring
 *               mass, and disk_mass is the sphere's mass (kg). Requires
 *               scheme 0, gravity_y = 0 (gravity across the axis breaks the
 *               symmetry) and audit = 0; the reverse sweep rejects it. */
typedef struct {
  double L, W, dx, h_over_dx, cell_size;
  double rho0, c0, gamma, p_cav;
  double alpha, delta, eps_xsph, mu_dyn, eta2;
  double cfl, gravity_y;
  double rho_lo, rho_hi, eps_wall;
  int ghost_layers, n_disk_ghosts, ghost_rho_mode, init_mode;
  double disk_R, disk_x0, disk_y0, disk_mass;
  int n_probes;
  double probe_xy[2 * WCSPH_MAX_PROBES];
  int diag_every;
  int kin_mode;
  double kin_v0, kin_t_ramp, kin_coef;
  int audit;
  double beta;
  int kernel_type;
  int eos_type;
  double mg_s1, mg_gamma0, mg_mu_max;
  int scheme;
  double mg_a;
  int axisym;
} wcsph_params;

/* One diagnostic record (FP64 reductions over the fluid of one instance).
 * ke, e_el (Tait elastic energy with the cutoff branch), e_pot (gravity),
 * e_disk = disk_mass v_d^2 / 2, w_boundary = integrated work of the disk
 * ghosts on the fluid (eq. energy-audit), n_clamp / n_enforce = cumulative
 * density-band and enforcement hits, n_cav = particles at the cutoff now.
 * Energy audit (audit = 1, else 0), integrals since the set-up, J per unit
 * depth: d_av and d_visc = irreversible dissipation of the artificial and
 * laminar viscosity between fluid particles (the D of eq. energy-audit),
 * w_delta = elastic energy rate of the delta diffusion, w_ghost = fluid
 * energy rate of every fluid-ghost pair term (walls and ring), all from the
 * midpoint rates times dt; w_enforce and w_clamp = energy the corrector's
 * enforcement and density clamp change. The change of ke + e_el + e_pot
 * equals w_ghost - d_av - d_visc + w_delta + w_enforce + w_clamp up to the
 * midpoint rule across enforcement and cutoff events (about 1 %). */
typedef struct {
  double t, dt, vmax, mass, mom[2], ke, e_el, e_pot, e_disk, w_boundary;
  long long step, n_clamp, n_cav, n_enforce;
  double d_av, d_visc, w_delta, w_ghost, w_enforce, w_clamp;
  double e_th; /* scheme 1: sum of m e, the internal energy (0 in scheme 0) */
} wcsph_diag;

typedef struct {
  int n_inst;          /* instances in the context (1 unless batched) */
  long long n_fluid;   /* fluid particles over all instances */
  long long n_ghost;   /* wall + disk ghosts over all instances */
  long long n_slots;   /* particles stored (fluid + ghosts) */
  long long n_cells;   /* cells over all instances */
  long long steps;     /* completed steps */
} wcsph_info;

/* ---- life cycle ---------------------------------------------------------- */

/* Build the initial state of the paper's problem set-up (Validation Problem
 * Setup; fluid lattice at ((i+1/2)dx, (j+1/2)dx) with the disk interior
 * removed, wall ghosts continuing the lattice ghost_layers deep, disk ring)
 * and capture one step as a HIP graph on `stream`.
 * alloc: NULL -> hipMalloc/hipFree. stream: a hipStream_t, not NULL.
 * Errors: E_INVALID (dx <= 0, h_over_dx outside [1,2], cell_size < 2h,
 * disk outside the box, n_probes > 16, ...) before any allocation;
 * E_OOM / E_HIP afterwards (the partially built context is released). */
wcsph_status wcsph_create(const wcsph_params* p, const wcsph_allocator* alloc, void* stream,
                          wcsph_ctx** out);

/* Batched coefficient sweep: n_inst independent instances (params[k] each,
 * sizes may differ) advanced together by the same kernels; every launch
 * covers all instances, with per-instance time step, clock and probes. */
wcsph_status wcsph_batch_create(const wcsph_params* params, int n_inst,
                                const wcsph_allocator* alloc, void* stream, wcsph_ctx** out);

wcsph_status wcsph_destroy(wcsph_ctx* ctx);
const char* wcsph_last_error(const wcsph_ctx* ctx);
wcsph_status wcsph_get_info(const wcsph_ctx* ctx, wcsph_info* out);
/* Per-instance sizes: fluid, ghosts (walls + ring), cells. */
wcsph_status wcsph_instance_info(const wcsph_ctx* ctx, int inst, int* n_fluid, int* n_ghost,
                                 int* n_cells);

/* ---- driving --------------------------------------------------------------- */

/* Disk kinematics of instance `inst` (Velocity Ramp, Projectile Dynamics).
 * mode 0: coeffs = {v0, t_ramp, a_d}; mode 1: {v0, t_ramp, k}; mode 2
 * (two-way coupling, see kin_mode): {v0, t_ramp, unused}; n = number of
 * coefficients (3). mode 3: a tabulated prescribed motion, coeffs = n rows
 * (t, x, v, a) row-major (1 <= n <= 1024, t strictly increasing, x the
 * centre's absolute position along the channel); each column is linear in t
 * between rows, and before the first row and after the last the centre moves
 * on at that row's velocity with zero acceleration. The table is copied to
 * the device (a context created with kin_mode 3 holds the disk at rest at
 * disk_x0 until a table is set). Takes effect at the next step, from the
 * disk state the new law gives at the newest state's time: a coupled disk is
 * released and a mode-2 disk couples again at its next step at or after
 * t_ramp. */
wcsph_status wcsph_set_disk_kinematics(wcsph_ctx* ctx, int inst, int mode, const double* coeffs,
                                       int n);

/* Fixed time-step table: when n > 0, step k (counted from the current
 * state) uses dt[k] for every instance instead of the CFL gate; n = 0
 * returns to the CFL gate. The table is copied. */
wcsph_status wcsph_set_dt_table(wcsph_ctx* ctx, const double* dt, int n);

/* Advance every instance by n_steps predictor-corrector steps (asynchronous
 * on the context stream). Each step: kinematics, cell list (stable sort by
 * cell key), Adami ghosts, probes, CFL step, pair sums + predictor; then the
 * same at the midpoint state + corrector (Pipeline Provenance section).
 * A diagnostic record is taken every diag_every steps. */
wcsph_status wcsph_step(wcsph_ctx* ctx, int n_steps);
/* The same for a batched context (wcsph_batch_create): every instance advances
 * n_steps steps, each kernel launched once for all instances. E_INVALID on a
 * single-instance context (wcsph_step serves both). */
wcsph_status wcsph_batch_step(wcsph_ctx* ctx, int n_steps);
wcsph_status wcsph_synchronize(wcsph_ctx* ctx);

/* ---- reading results ------------------------------------------------------- */

/* Probe history of instance `inst` since the last read: per step n, the time
 * t_n, the step dt_n and n_probes pressures (row-major). The device ring holds
 * the last 65536 steps; older rows are dropped.
 *
 * Validity: this reader, wcsph_get_fluid, wcsph_get_disk, wcsph_adj_forward
 * and wcsph_adj_backward return E_UNSTABLE, after writing their outputs, when
 * the device state carries a validity flag (a non-finite value or escaped
 * particle, a cell with more than 64 particles or a broken permutation);
 * wcsph_last_error names the flags. */
wcsph_status wcsph_read_probes(wcsph_ctx* ctx, int inst, double* t, double* dt, float* p,
                               int max_rows, int* rows_out);
/* Diagnostic records of instance `inst` since the last read (ring of 4096).
 * Returns E_UNSTABLE (records still written) if a record found a non-finite
 * value or the cell list broke down (a cell with more than 64 particles);
 * wcsph_last_error names which. */
wcsph_status wcsph_read_diagnostics(wcsph_ctx* ctx, int inst, wcsph_diag* out, int max, int* n_out);

/* Fluid state of instance `inst` in particle-id order (id = j nx + i of the
 * lattice, disk interior skipped), decoded to FP64; n = its fluid count. */
wcsph_status wcsph_get_fluid(wcsph_ctx* ctx, int inst, double* t, double* x, double* y, double* vx,
                             double* vy, double* rho, int n);
/* Scheme 1: specific internal energy e (J/kg) of instance `inst` in
 * particle-id order (zero in scheme 0); n = its fluid count (E_RANGE if
 * smaller). Same validity rule as wcsph_get_fluid. */
wcsph_status wcsph_get_internal_energy(wcsph_ctx* ctx, int inst, double* e, int n);
/* Disk centre x, velocity and acceleration (along +x) of instance `inst` at
 * the newest state's time (any pointer may be NULL). For a coupled disk the
 * acceleration is that of the last step. Synchronises the context stream. */
wcsph_status wcsph_get_disk(wcsph_ctx* ctx, int inst, double* x, double* v, double* a);

/* Replace the fluid state of every instance (single-instance contexts only):
 * positions are encoded as (cell, FP32 offset), velocities and density to
 * FP32; storage order is reset to id order and the clock set to t (scheme 1:
 * the internal energy to zero, the previous step to none). */
wcsph_status wcsph_set_fluid(wcsph_ctx* ctx, double t, const double* x, const double* y,
                             const double* vx, const double* vy, const double* rho, int n);

/* Opaque checkpoint of the whole device state (clock, encoded particles,
 * storage order). need returns the size; cap too small -> E_RANGE. */
wcsph_status wcsph_save_state(wcsph_ctx* ctx, void* buf, size_t cap, size_t* need);
wcsph_status wcsph_load_state(wcsph_ctx* ctx, const void* buf, size_t n);

/* ---- test hooks -------------------------------------------------------------- */

/* One cell-list build on the current state (single instance): per slot of
 * the pre-sort order the key, particle id and decoded position; the stable
 * permutation perm[new] = old; the ids in sorted order; cell_start[ncells+1].
 * The state is left unchanged. */
wcsph_status wcsph_export_cells(wcsph_ctx* ctx, unsigned* keys, unsigned* ids_pre, double* x,
                                double* y, unsigned* perm, unsigned* ids_post, unsigned* cell_start,
                                size_t cap_slots, size_t cap_cells);
/* One evaluation on the current state (ghosts then pair sums, single
 * instance): density rate, acceleration and XSPH velocity per fluid id, ghost
 * pressure / density / velocity per ghost index (walls then ring). Scheme 1
 * (summed density first): drho holds the internal-energy rate de/dt. */
wcsph_status wcsph_export_rates(wcsph_ctx* ctx, float* drho, float* ax, float* ay, float* Vx,
                                float* Vy, float* gp, float* grho, float* gvx, float* gvy,
                                int n_fluid, int n_ghost);
/* Density and pressure of every fluid particle at the current state, by
 * fluid id (single instance): scheme 0 the stored density and its EOS
 * pressure; scheme 1 the clamped summation (eq. density-sum) at the current
 * positions and the pressure with the internal energy. The state is left
 * unchanged. n_fluid smaller than the fluid count -> E_RANGE. */
wcsph_status wcsph_export_density(wcsph_ctx* ctx, float* rho, float* p, int n_fluid);
/* In-support neighbour count and neighbour-id sum per particle (ids in
 * sorted order), plus decoded positions; single instance. */
wcsph_status wcsph_export_neighbours(wcsph_ctx* ctx, unsigned* ids, int* count, long long* idsum,
                                     double* x, double* y, size_t cap_slots);
/* The in-support neighbours of every fluid particle as the pair-sum kernel
 * of one evaluation on the current state finds them (single instance):
 * count[k] and the ids nbr[k * max_per + i], i < count[k], of fluid
 * particle k, in no particular order (ids: fluid, then wall ghosts, then
 * ring ghosts). The state is left unchanged. E_RANGE if a
 * particle has more than max_per (or 64) neighbours. */
wcsph_status wcsph_export_neighbour_lists(wcsph_ctx* ctx, int* count, unsigned* nbr, int max_per,
                                          int n_fluid);
/* The same lists without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid it). The export buffer is a file-scope device array
 * of 4 MiB that each GPU the library runs on holds until the process ends;
 * it fits a context of at most 16,131 fluid particles (E_RANGE beyond, with
 * nothing run). Calls share their GPU's array: calls that overlap on one GPU
 * race. Same outputs and errors as wcsph_export_neighbour_lists; calls no
 * allocator. */
wcsph_status wcsph_export_neighbour_lists_noalloc(wcsph_ctx* ctx, int* count, unsigned* nbr, int max_per,
                                                  int n_fluid);
/* Measurement hook: average duration (ms) of the pair-sum kernel of the
 * first evaluation, re-launched `reps` (1..1000) times back to back on the
 * current sorted state between two HIP events on the context stream. The
 * state is restored. */
wcsph_status wcsph_time_pair_kernel(wcsph_ctx* ctx, int reps, float* avg_ms);

/* ---- coefficients and reverse sweep --------------------------------------- */

/* Replace the Monaghan alpha, the delta-diffusion coefficient and the Tait
 * sound speed c0 of instance `inst` (B = rho0 c0^2 / gamma and every constant
 * derived from them follow). The particle state is untouched. */
wcsph_status wcsph_set_coefficients(wcsph_ctx* ctx, int inst, double alpha, double delta, double c0);

/* Reverse-mode gradient of the summed wall-probe pressure impulse
 *   J = sum_k sum_n p_k^n dt_n   (probes sampled at the state of step n)
 * with respect to (alpha, delta, c0), for a single-instance context with the
 * linear ghost density, the rest initial state, a prescribed disk motion
 * (kin_mode 0 or 1) and the linear artificial viscosity (beta = 0), at a
 * fixed time-step table (wcsph_set_dt_table must
 * cover the run, so dt does not depend on c0).
 * adj_forward advances n_steps from the current state, keeps a device
 * checkpoint every ckpt_every steps and returns J. With ckpt_every >=
 * n_steps (and no energy audit) the forward itself tapes every evaluation
 * (about 2 * (40 n_slots + 32 n_fluid) bytes per step, one allocation, kept
 * for later calls) and the backward replays nothing; the tape is bitwise
 * that of a replay. Otherwise adj_backward walks the
 * segments last to first: it restores a checkpoint, replays the segment
 * taping each evaluation's sorted state and pre-enforcement state. It runs
 * the hand-written transpose of the step (enforcement, pair sums, Adami ghost
 * Shepard sums, probes, Tait EOS) in FP32 with FP64 coefficient
 * accumulators; grad[3] = dJ * dJ/d(alpha, delta, c0). The state is left at
 * the end of the forward run. Non-smooth points (AV switch, cavitation
 * cutoff, density band, enforcement) take the branch of the forward run. */
wcsph_status wcsph_adj_forward(wcsph_ctx* ctx, int n_steps, int ckpt_every, double* J);
wcsph_status wcsph_adj_backward(wcsph_ctx* ctx, double dJ, double* grad);

#ifdef __cplusplus
}
#endif
#endif /* WCSPH_H */
