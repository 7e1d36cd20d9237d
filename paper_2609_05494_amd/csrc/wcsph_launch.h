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

void wc_enqueue_step(const Dev& d, const Bufs& b, int n_gblk, bool batch, hipStream_t st);
void wc_enqueue_init(const Dev& d, const Bufs& b, bool batch, hipStream_t st);
void wc_enqueue_diag(const Dev& d, const Bufs& b, int row, bool sorted, hipStream_t st);
void wc_enqueue_export_sort(const Dev& d, const Bufs& b, bool batch, hipStream_t st);
void wc_enqueue_export_ghosts(const Dev& d, const Bufs& b, int n_gblk, hipStream_t st);
void wc_enqueue_export_pair(const Dev& d, const Bufs& b, hipStream_t st);
void wc_enqueue_pair_a(const Dev& d, const Bufs& b, bool batch, hipStream_t st);
void wc_enqueue_neigh(const Dev& d, const Bufs& b, hipStream_t st);
