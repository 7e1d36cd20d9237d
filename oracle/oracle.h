/*
 * oracle.h -- C interface of the FP64 CPU oracle of the planar WCSPH step.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the plain, slow reference the
 * GPU path is checked against. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. It shares no code with the
 * GPU library.
 *
 * Units are SI throughout. Positions are metres in the frame where the fluid
 * box is [0,L]x[0,W]. All arrays are caller-owned; sizes are stated per call.
 */
#ifndef WCSPH_ORACLE_H
#define WCSPH_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_PROBES 16
/* t dt vmax mass momx momy ke e_el e_pot e_disk w_boundary step n_clamp n_cav n_enforce
 * d_av d_visc w_delta w_ghost w_enforce w_clamp (energy audit integrals, J per unit depth)
 * e_th (sum of m e, the internal energy of scheme 1) */
#define ORC_NDIAG 22

typedef struct {
  double L, W, dx, h_over_dx, cell_size;  /* cell_size <= 0 -> 2h */
  double rho0, c0, gamma, p_cav;
  double alpha, delta, eps_xsph, mu_dyn, eta2;
  double cfl, gravity_y;
  double rho_lo, rho_hi, eps_wall;         /* density band in units of rho0 */
  int ghost_layers, n_disk_ghosts, ghost_rho_mode, init_mode;
  double disk_R, disk_x0, disk_y0, disk_mass;
  int n_probes;
  double probe_xy[2 * ORC_MAX_PROBES];
  int diag_every;
  int kin_mode; /* 0: ramp then constant deceleration kin_coef; 1: ramp then quadratic drag k=kin_coef;
                  2: ramp then two-way coupling; 3: tabulated (orc_set_kin_table) */
  double kin_v0, kin_t_ramp, kin_coef;
  double beta; /* quadratic artificial viscosity coefficient (0: linear term only) */
  int kernel_type; /* 0: Wendland C2; 1: cubic B-spline (eq. cubic-kernel) */
  int eos_type;    /* 0: Tait; 1: Mie-Grueneisen of eq. eos at zero specific internal energy */
  double mg_s1, mg_gamma0, mg_mu_max; /* its Hugoniot slope S1, gamma0 and compression cap */
  int scheme;  /* 0: continuity + delta term, predictor-corrector;
                  1: the paper as published: summation density (eq. density-sum, ghosts in
                  the sum, lattice-normalised masses) with its clamp, leapfrog, and the
                  specific internal energy heated by the artificial viscosity */
  double mg_a; /* the a of eq. eos (scheme 1 with eos_type 1) */
  int axisym;  /* 1: the axisymmetric r-z form (the extension the Conclusions rank first): x is the
                  axial coordinate z, y >= 0 the radius r, the box's y = 0 edge the symmetry axis;
                  fluid particles carry fixed ring masses 2 pi r0 rho0 dx^2, continuity gains the
                  hoop term -rho v_r / r, the ghost layers below the axis mirror the fluid (slip)
                  and are off inside the sphere; needs scheme 0 and gravity_y = 0 */
} orc_params;

/* ---- whole solver ------------------------------------------------------ */
/* init: NULL -> lattice set-up of the paper; else n_init rows of (x,y,vx,vy,rho). */
void* orc_create(const orc_params* p, int n_init, const double* init);
void orc_destroy(void* s);
int orc_num_fluid(void* s);
int orc_num_ghost(void* s);
int orc_num_cells(void* s);
/* dt table: if n > 0, step k uses dt[k] instead of the CFL gate. */
void orc_set_dt_table(void* s, int n, const double* dt);
int orc_step(void* s, int n_steps);
void orc_get_fluid(void* s, double* t, double* x, double* y, double* vx, double* vy, double* rho);
/* replace the fluid state; resets the storage order to id order */
void orc_set_fluid(void* s, double t, const double* x, const double* y, const double* vx,
                   const double* vy, const double* rho);
int orc_probe_rows(void* s);
void orc_get_probes(void* s, double* t, double* dt, double* p /* rows x n_probes */);
int orc_diag_rows(void* s);
void orc_get_diags(void* s, double* rows /* rows x ORC_NDIAG */);
double orc_impulse(void* s); /* J = sum_k sum_n p_k^n dt_n */
/* one evaluation at the current state and time (ghosts, then rates), by fluid
 * id; ghost outputs by ghost index (walls first, then disk). Leaves the state
 * untouched except for the storage order. */
void orc_eval_rates(void* s, double* drho, double* ax, double* ay, double* Vx, double* Vy,
                    double* gp, double* grho, double* gvx, double* gvy, double* vmax);
/* Energy audit rates of the last rate evaluation (J/s per unit depth):
 * D_av' and D_visc' (fluid pairs, >= 0), W_delta', W_ghost' (every
 * fluid-ghost pair term). For any state, sum_i m_i (v_i.a_i + P_i drho_i
 * - v_i.g) = W_ghost' - D_av' - D_visc' + W_delta'. */
void orc_audit_rates(void* s, double* out /* 4 */);
void orc_get_ghosts(void* s, double* gx, double* gy, double* gm);
/* Fluid density and pressure by fluid id at the current state: scheme 0 the
 * stored density; scheme 1 the clamped summation over fluid and ghosts at
 * the current positions (disk ring at the current time), which is stored.
 * Pressure with the cutoff and, scheme 1, the internal energy. */
void orc_eval_density(void* s, double* rho, double* p);
/* specific internal energy by fluid id (scheme 1; zero otherwise) */
void orc_get_energy(void* s, double* e);
/* pressure of eq. eos with the cutoff at density rho and specific internal energy e */
double orc_eos_pe(const orc_params* p, double rho, double e);
/* the lattice-normalised particle mass of scheme 1: rho0 / sum_j W(r_j) over
 * the points r_j = (i dx, j dx) in support */
double orc_lattice_mass(const orc_params* p);
void orc_get_order(void* s, int* order, int* cell_start);
void orc_kinematics(void* s, double t, double* x, double* v, double* a);
/* kin_mode 3: the prescribed disk motion as n rows (t, x, v, a), t strictly
 * increasing, x the centre's absolute position; each column is interpolated
 * linearly between rows, and outside the table the centre moves on at the
 * end row's velocity with zero acceleration. */
void orc_set_kin_table(void* s, int n, const double* rows);
// disk centre x, velocity, acceleration at the current time (kin_mode 2:
// the coupled state once the first step after the ramp has started)
void orc_disk_state(void* s, double* x, double* v, double* a);

/* ---- building blocks (exposed for the pin tests) ------------------------ */
void orc_kernel(double q, double h, double* W, double* F);
/* Kernel of type 0 (Wendland C2) or 1 (cubic B-spline): W and F = (1/r) dW/dr. */
void orc_kernel_type(int type, double q, double h, double* W, double* F);
void orc_eos(const orc_params* p, double rho, double* pres, double* c);
/* Density at pressure pres >= p_cav on the EOS of p (its inverse, no cutoff branch). */
double orc_eos_rho(const orc_params* p, double pres);
double orc_elastic_energy(const orc_params* p, double rho);
double orc_cfl_dt(double cfl, double h, double c0, double vmax);
/* Cell list of n points given in current storage order: keys[k] of slot k,
 * perm[new slot] = old slot (stable), cell_start[ncells+1]. Returns ncells. */
int orc_cell_list(const orc_params* p, int n, const double* x, const double* y, int* keys,
                  int* perm, int* cell_start);
/* number of pairs (i<j) with |r_ij| < 2h by O(N^2) search / via the cell list;
 * pairs written as (i,j) if out != NULL (capacity cap pairs). */
long orc_brute_pairs(const orc_params* p, int n, const double* x, const double* y, int* out, long cap);
long orc_cell_pairs(const orc_params* p, int n, const double* x, const double* y, int* out, long cap);
/* per point: in-support neighbour count, sum of neighbour ids, count of pairs
 * with |r^2 - 4h^2| < tol*4h^2 (the borderline pairs). */
void orc_neighbour_stats(const orc_params* p, int n, const double* x, const double* y,
                         const int* ids, double tol, int* count, long long* idsum, int* border);
/* Adami-Shepard ghost state at point (gx,gy) with wall velocity vw and
 * acceleration aw, over nf fluid points (brute force). */
void orc_ghost_point(const orc_params* p, double gx, double gy, const double* vw, const double* aw,
                     int nf, const double* x, const double* y, const double* vx, const double* vy,
                     const double* rho, const double* pres, double* pg, double* rhog, double* vg);
/* Pair-sum rates over an arbitrary particle set by brute force; kind[j] = 0
 * fluid, 1 wall ghost, 2 disk ghost; for ghosts pres[] is p_g and rho[] is
 * rho_g. Rates are written for fluid entries only. */
void orc_pair_rates(const orc_params* p, int n, const double* x, const double* y, const double* vx,
                    const double* vy, const double* rho, const double* pres, const double* m,
                    const int* kind, double* drho, double* ax, double* ay, double* Vx, double* Vy);

/* ---- forward-mode tangent (dual numbers in alpha, delta, c0) ------------- */
/* Runs n_steps from the set-up state with the given dt table and returns
 * J and dJ/d(alpha, delta, c0). */
void orc_tangent_J(const orc_params* p, int n_steps, const double* dt, double* J, double* dJ);
/* The same with the state's values rounded to the FP32 representation of the
 * hot path after every step (cell + float32 offset, float32 v and rho; the
 * tangents are kept): how far FP32 storage alone moves J and its gradient. */
void orc_tangent_J_f32(const orc_params* p, int n_steps, const double* dt, double* J, double* dJ);

#ifdef __cplusplus
}
#endif
#endif
