// wcsph_dev.h -- device-side data layout shared by the kernels and the host
// runtime of libwcsph.so (internal; not part of the C ABI).
//
// Particles (fluid, wall ghosts, disk ghosts of every instance) live in one
// slot space. Each buffer is a structure of arrays in slot order; after a
// sort the slots are ordered by global cell key, so the particles of a cell
// (and of an instance) are contiguous. Positions are encoded as the cell key
// plus an FP32 offset inside the cell, so pair distances are formed from
// cell-relative coordinates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define WC_MAX_PROBES 16
#define WC_HIST_CAP 65536
#define WC_DIAG_CAP 4096
#define WC_NDIAG 22
#define WC_BLOCK 256
#define WC_GHOST_BLOCK 256
#ifndef WC_GHOST_LANES
#define WC_GHOST_LANES 16      // lanes per ghost or probe in the ghost kernel
#endif
#define WC_MAX_RING 256        // disk-ring ghosts per instance
#define WC_DIAG_BLOCKS 256     // diagnostic partial sums per instance
#define WC_BUCKET 64           // capacity of one cell bucket (particles per cell)
#define WC_SORT_TILE 64        // cells per block of the sort kernel
#define WC_NB_CAP 64           // neighbour ids per particle in the neighbour-list export
#define WC_KIN_ROWS 1024       // rows of a tabulated disk motion per instance
#define WC_NO_ID 0xffffffffu   // particle id of an inert sorted entry (a gap left by a bucket overflow)

// Per-instance constants (read-only in kernels).
struct InstParams {
  // grid: cell key = cell_off + cy * ncx + cx; origin (x_lo, y_lo); edge dc
  double x_lo, y_lo, dcd, inv_dcd;
  float dc;
  int ncx, ncy, cell_off, ncell;
  // ids: [id0, id0+nf) fluid, then nw wall ghosts, then nd disk ghosts;
  // ghost g of this instance is tracked at gslot[gmap0 + g]
  int id0, nf, nw, nd, gmap0;
  // pair arithmetic (FP32)
  float h, inv_h, four_h2, sigma, fgrad, eta2h2;
  float rho0, c0, B, p_cav, alpha, eps_xsph, gy;
  float beta2h2;  // 2 beta h^2: quadratic AV term beta mu^2 / rho_bar (0: linear term only)
  int kernel_type;       // 0 Wendland C2, 1 cubic B-spline
  float kc_sigma, kc_a;  // cubic spline: 10 / (7 pi h^2) and that over h^2
  float two_delta_h_c0, four_nu0, delta, two_h_c0;
  float m_fluid, m_wall, m_disk;
  float rho_lo, rho_hi, inv_rho0c02, c_exp, gamma, inv_gamma;
  int ghost_rho_mode;
  // FP64 geometry, kinematics and step control
  double L, W, eps_wall, R, disk_x0, disk_y0, disk_mass, cfl, hd, c0d, Bd, rho0d, gammad, p_cavd;
  double m_fluidd;  // rho0 dx^2 for the FP64 diagnostics
  // FP64 constants of the Tait elastic energy (diagnostics): cutoff density,
  // B / ((gamma - 1) rho0^gamma), rho0^(gamma - 1), energy at the cutoff,
  // rho0^-gamma
  double diag_rc, diag_k1, diag_r0g1, diag_erc, diag_inv_r0g;
  int kin_mode;
  double kin_v0, kin_t_ramp, kin_coef;
  // probes: encoded positions
  int n_probes;
  uint32_t probe_cell[WC_MAX_PROBES];
  float probe_ox[WC_MAX_PROBES], probe_oy[WC_MAX_PROBES];
  // EOS (kept last: the fields above keep their offsets): 0 Tait; 1 the Mie-Grueneisen law at zero internal energy, with
  // K = rho0 C^2 (C = c0), k1 = 1 - gamma0/2, b = S1 - 1 and the cap of mu
  int eos_type;
  float mg_K, mg_k1, mg_b, mg_mu_max;
  // the same law in FP64 (diagnostics): K, k1, b, the cap, mu at the cutoff
  // p_cav / K and the pressure at the cap
  double mg_Kd, mg_k1d, mg_bd, mg_mu_maxd, mg_mu_cavd, mg_p_capd;
  // kin_mode 3: the instance's table of prescribed motion, kin_tab_n rows (t, x, v, a) (device)
  const double* kin_tab;
  int kin_tab_n;
  // scheme 0: continuity + delta term, predictor-corrector; 1: the paper as
  // published (summation density over fluid and ghosts with the density
  // band, leapfrog, the specific internal energy heated by the artificial
  // viscosity, and with the Mie-Grueneisen law its energy term (gamma0 +
  // mg_a mu) rho e). Scheme 1 masses are lattice-normalised (m_fluid etc.).
  int scheme;
  float mg_a, mg_g0;
  double mg_ad, mg_g0d;
  // axisymmetric r-z form: x axial, y the radius from the axis y = 0; the
  // radius below which the hoop term and the planar ring mass hold (dx/2)
  int axisym;
  float r_min;
  double r_mind;
};

// Per-instance clock and accumulators (device-resident, FP64 time).
struct Clock {
  double t;        // time of the current step's state n
  double t_next;   // t + dt once the step has completed (the time of the newest state)
  double dt;       // dt of the current step
  double t_eval;   // time of the current evaluation
  double xd, vd, ad;  // disk centre x, velocity, acceleration at t_eval
  double xd_next, vd_next;  // disk centre x and velocity at t + dt (from the second evaluation on)
  double ac_next;     // coupled disk: acceleration over the step (the state at t + dt)
  double xc, vc, ac;  // coupled disk: centre x, velocity, latest acceleration at t
  double v_work;      // coupled disk: mean velocity of the step (boundary work)
  double w_boundary;  // integrated work of the disk ghosts on the fluid
  double vmax_used;   // v_max that set dt
  double dt_prev;     // scheme 1: dt of the previous step (0 before the first), for the merged kick
  long long step;     // index of the current step (-1 before the first)
  long long diag_row; // diagnostic records written so far
  unsigned long long n_clamp, n_enforce;
  unsigned int vmax_bits;  // running max of |v| (float bits) for the next dt
  unsigned int bad;        // non-finite / escaped-particle flag
  int coupled;             // kin_mode 2: the disk moves under the fluid force (from the step at t >= t_ramp)
  int pad_;
};

// One particle buffer (structure of arrays in slot order).
struct Buf {
  uint32_t* cell;   // global cell key
  uint32_t* id;     // global particle id
  float4* pv;       // (ox, oy, vx, vy): offset inside the cell, velocity
  float4* aux;      // (rho, P = p / rho^2, c, m) ; m < 0 marks a ghost
  uint16_t* inst;   // instance (batched contexts only)
  float* e;         // scheme 1: specific internal energy (NULL otherwise)
};

// Everything a kernel may touch (passed by value).
struct Dev {
  const InstParams* prm;
  Clock* clk;
  int n_inst, n_slots, n_cells, n_ghost;
  uint32_t* count;            // per cell: bucket fill for the next sort
  uint32_t* start;            // per cell + 1: exclusive scan of count
  const uint32_t* wallcount;  // per cell: static wall ghosts (pre-fill of count)
  // cell buckets [n_cells][WC_BUCKET] of slots, filled for the next sort:
  // bucket_a by eval B (and at load) for eval A, bucket_b by eval A for eval B
  uint32_t* bucket_a;
  uint32_t* bucket_b;
  // entries per sort tile of the bucket set a / b, filled with the buckets;
  // the static wall-ghost entries they are re-armed with
  uint32_t* tot_a;
  uint32_t* tot_b;
  const uint32_t* wall_tot;
  uint32_t* perm;             // per slot: perm[new] = old of the last sort
  const double2* ring_cs;     // [n_inst][WC_MAX_RING] (cos, sin) of the ring angles
  uint32_t* gslot;            // per ghost: current slot
  uint32_t* gcell;            // per ghost: cell key in the current sorted order
  float2* gpos;               // per ghost: offset inside that cell
  const uint32_t* wrank;      // per ghost: static bucket rank of a wall ghost
  const int4* gblk;           // ghost-kernel block table: (inst, first item, count, kind)
  double* hist_t;             // [n_inst][WC_HIST_CAP]
  double* hist_dt;
  float* hist_p;              // [n_inst][WC_HIST_CAP][WC_MAX_PROBES]
  const double* dt_table;     // fixed steps (dt_mode), n_dt entries from step dt_step0
  int n_dt;
  long long dt_step0;
  double* diag;               // [n_inst][WC_DIAG_CAP][WC_NDIAG]
  double* diag_part;          // [n_inst][WC_DIAG_BLOCKS][WC_DIAG_PARTS] partial sums
  double* wb_part;            // [n_inst][WC_MAX_RING] x force of each ring ghost on the fluid
  float* vmax_part;           // single instance: per corrector pair wave, max |v| of its new fluid
                              // state (folded into the clock by the next first-evaluation sort)
  int n_vpart;                // entries of vmax_part and audit_part (waves of the pair pass)
  int var;                    // pass variants: bit 0 quadratic AV (some beta > 0), bit 1 cubic spline,
                              // bit 2 some instance uses the Mie-Grueneisen EOS (sort pass)
  int lf_set;                 // scheme 1: the bucket set (0 a, 1 b) this step's sort reads; its
                              // pair pass fills the other
  double* audit_part;         // energy audit (single instance, or NULL): per corrector pair wave,
                              // running sums of d_av, d_visc, w_delta, w_ghost, w_enforce, w_clamp
  float* xr;                  // export: [5][n_slots] rates per slot
  int* nb_count;              // export: neighbour count per slot
  long long* nb_idsum;        // export: neighbour id sum per slot
  uint32_t* nb_ids;           // export: per fluid index, neighbour count [nf], then ids [nf][WC_NB_CAP] (or NULL)
  const double* mring;        // axisymmetric instances: ring mass per radian M / (2 pi) by particle id
                              // (fluid ids; NULL when no instance is axisymmetric)
  double2* tape_pos;          // reverse sweep: pre-enforcement position per fluid id (or NULL)
  float4* tape_vel;           // reverse sweep: pre-enforcement (vx, vy, rho, 0) per fluid id
};

// One taped evaluation for the reverse sweep: the sorted state (with ghost
// states), its cell ranges and ghost slots.
struct TapeEval {
  uint32_t* cell;
  uint32_t* id;
  float4* pv;
  float4* aux;
  uint32_t* start;
  uint32_t* gslot;
};

// Reverse-sweep work arrays (adjoints by fluid id unless stated).
struct AdjPtrs {
  float* lam_out;      // [5][nf] adjoint of the evaluation's output state (x, y, vx, vy, rho)
  float* lam_base;     // [5][nf] adjoint of the base / evaluated state
  float* lam_s;        // rate adjoints in sorted slot order: float4 (D, ax, ay, Vx) [n_slots], then Vy [n_slots]
  float* gadj;         // [n_slots][10] ghost adjoint and Shepard data
  float* padj;         // [16][2] probe Shepard sums
  double2* pre_pos;    // taped pre-enforcement state of the evaluation
  float4* pre_vel;
  double* theta_part;  // per-block running sums of the coefficient gradients over the sweep [blocks][3]
  double* theta;       // dJ/d(alpha, delta, c0), FP64
  int n_ghost_probe;
};

// Passes: EV_A / EV_B the predictor / corrector evaluation, EV_EXPORT an
// evaluation of the newest state that changes nothing (test hooks), EV_L the
// single evaluation of a scheme-1 (leapfrog) step.
enum { EV_A = 0, EV_B = 1, EV_EXPORT = 2, EV_L = 3 };
#define WC_DIAG_PARTS 9  // M, px, py, ke, e_el, e_pot, n_cav, bad, e_th


