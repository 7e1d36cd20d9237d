// wcsph_launch.h -- host entry points of the kernels translation unit
// (internal to libwcsph.so).
#pragma once

#include "wcsph_dev.h"

// The four particle buffers of a step: X holds state n (and after the step
// state n+1), Y the sorted state n, Z the predicted state, W the sorted
// predicted state.
struct Bufs {
  Buf X, Y, Z, W;
};

// two_way: some instance has a two-way coupled disk (kin_mode 2)
// audit: single-instance energy audit in the second pair pass
void wc_enqueue_step(const Dev& d, const Bufs& b, int n_gblk, bool batch, bool two_way, bool audit,
                     hipStream_t st);
// Disk centre, velocity, acceleration of instance inst's newest state into out[3] (device).
// One leapfrog step (scheme 1) whose sort reads bucket set `set` (0 a, 1 b);
// its pair pass fills the other set.
void wc_enqueue_step_lf(const Dev& d, const Bufs& b, int n_gblk, bool batch, int set, hipStream_t st);
// Summation density and EOS in place on the export sort's state (scheme 1).
void wc_enqueue_export_dens(const Dev& d, const Bufs& b, hipStream_t st);
void wc_enqueue_disk_query(const Dev& d, int inst, double* out, hipStream_t st);
void wc_enqueue_init(const Dev& d, const Bufs& b, bool batch, hipStream_t st);
void wc_enqueue_diag(const Dev& d, const Bufs& b, bool sorted, hipStream_t st);
void wc_enqueue_export_sort(const Dev& d, const Bufs& b, bool batch, hipStream_t st);
void wc_enqueue_export_ghosts(const Dev& d, const Bufs& b, int n_gblk, hipStream_t st);
void wc_enqueue_export_pair(const Dev& d, const Bufs& b, hipStream_t st);
void wc_enqueue_pair_a(const Dev& d, const Bufs& b, bool batch, hipStream_t st);
void wc_enqueue_neigh(const Dev& d, const Bufs& b, hipStream_t st);

// One evaluation (A: sort of X into Y, ghosts, pair sums + predictor into Z;
// B: sort of Z into W with state n into X, ghosts, pair sums + corrector)
// with plain launches; single instance.
void wc_enqueue_eval(const Dev& d, const Bufs& b, int n_gblk, int mode, hipStream_t st);
// blocks of one pair-kernel launch over n_slots slots
int wc_pair_blocks(int n_slots);
// number of per-block theta partials one adjoint rate evaluation writes
int wc_adj_partial_blocks(int n_ghost_probe, int n_slots);
// The reverse of one evaluation: the enforcement transpose (adjoint
// pointers ae: lam_out -> lam_base, added when acc_enf; the rate adjoints
// into the taped slot order) in one launch with the ghost adjoints, then
// the fluid adjoints (pointers ar: into ar.lam_base, added when acc_rates;
// probe terms when probe_seed != 0).
void wc_enqueue_adj_eval(const Dev& d, const AdjPtrs& ae, const AdjPtrs& ar, const TapeEval& te, double t_enf,
                         float hdt, bool acc_enf, double t_eval, float probe_seed, bool acc_rates, hipStream_t st);
// theta += the per-block running sums of the coefficient partials (after the sweep)
void wc_enqueue_adj_theta(const AdjPtrs& a, int nblk, hipStream_t st);
