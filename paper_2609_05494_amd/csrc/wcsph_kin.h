// wcsph_kin.h -- the prescribed disk motion along +x, FP64, shared by the
// forward kernels and the reverse sweep of libwcsph.so (internal).
#pragma once

#include "wcsph_dev.h"

// Velocity ramp (eq. velocity-ramp) to v0 over t_ramp, then (kin_mode 0) the
// constant deceleration kin_coef until the disk stops, or (kin_mode 1) the
// quadratic drag of eq. drag with k = kin_coef, in closed form. kin_mode 2
// (two-way coupling) follows the ramp and then v0 until its first coupled
// step. kin_mode 3: the table of kin_tab_n rows (t, x, v, a), each column
// linear in t between rows (a row's own time gives the row); before the first
// row and after the last the centre moves on at that row's velocity with zero
// acceleration; an empty table holds the disk at rest at disk_x0.
__device__ inline void table_kinematics(const InstParams& P, double t, double& x, double& v, double& a) {
  const int n = P.kin_tab_n;
  const double* T = P.kin_tab;
  if (n <= 0) {
    x = P.disk_x0;
    v = 0.0;
    a = 0.0;
    return;
  }
  if (t < T[0]) {
    x = T[1] + T[2] * (t - T[0]);
    v = T[2];
    a = 0.0;
    return;
  }
  // the last row with t_k <= t (binary search)
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (T[4 * mid] <= t) lo = mid;
    else hi = mid;
  }
  const double* r = T + 4 * lo;
  if (lo == n - 1) {
    x = t == r[0] ? r[1] : r[1] + r[2] * (t - r[0]);
    v = r[2];
    a = t == r[0] ? r[3] : 0.0;
    return;
  }
  const double w = (t - r[0]) / (r[4] - r[0]);
  x = r[1] + w * (r[5] - r[1]);
  v = r[2] + w * (r[6] - r[2]);
  a = r[3] + w * (r[7] - r[3]);
}

__device__ inline void kinematics(const InstParams& P, double t, double& x, double& v, double& a) {
  if (P.kin_mode == 3) {
    table_kinematics(P, t, x, v, a);
    return;
  }
  const double v0 = P.kin_v0, tr = P.kin_t_ramp;
  if (t < tr) {
    v = v0 * t / tr;
    a = v0 / tr;
    x = P.disk_x0 + 0.5 * v0 * t * t / tr;
    return;
  }
  const double tau = t - tr, xr = P.disk_x0 + 0.5 * v0 * tr;
  if (P.kin_mode == 2) {
    v = v0;
    a = 0.0;
    x = xr + v0 * tau;
    return;
  }
  if (P.kin_mode == 1) {
    const double k = P.kin_coef;
    v = v0 / (1.0 + k * v0 * tau);
    a = -k * v * v;
    x = k > 0.0 ? xr + log1p(k * v0 * tau) / k : xr + v0 * tau;
    return;
  }
  const double ad = P.kin_coef;
  if (ad > 0.0 && tau >= v0 / ad) {
    v = 0.0;
    a = 0.0;
    x = xr + 0.5 * v0 * v0 / ad;
    return;
  }
  v = v0 - ad * tau;
  a = -ad;
  x = xr + v0 * tau - 0.5 * ad * tau * tau;
}
