// wcsph_oracle.cpp -- FP64 CPU oracle of the planar WCSPH step.
//
// TEST INFRASTRUCTURE ONLY: the plain, slow, obviously correct reference the
// GPU path is checked against. Only the tests, the smoke check and the CPU
// baseline of the benchmark load it; it shares no code with the GPU library.
//
// What it computes, step by step, in the paper's order and notation
// (planar WCSPH model for hydrodynamic ram, Numerical Methodology section),
// with the scheme choices of the hot path where they differ from the paper:
//  * SPH interpolant with a compact kernel of support 2h, h = 1.3 dx
//    (eq. sph-approx); kernel = Wendland C2 in 2D instead of the paper's
//    cubic B-spline (eq. cubic-kernel), which kernel_type 1 selects.
//  * momentum in the symmetric form (eq. momentum) with the Monaghan
//    artificial viscosity (eq. artificial-viscosity; the linear term, plus
//    the quadratic beta mu^2 term the paper omits, off unless beta > 0), plus
//    a laminar term in the Lo-Shao form for the physical viscosity
//    (the viscosity paragraph of Governing Equations).
//  * XSPH-smoothed advection velocity over fluid neighbours (eq. xsph).
//  * density from the continuity equation with the Molteni-Colagrossi
//    delta-diffusion term (named as the alternative in Density Summation),
//    clamped to the band [0.5, 1.5] rho0 after every update.
//  * Tait EOS p = B((rho/rho0)^gamma - 1), B = rho0 c0^2 / gamma, with the
//    cavitation cutoff p >= p_cav (eq. eos text).
//  * predictor-corrector (explicit midpoint) update with the CFL step of
//    eq. cfl, v_max over fluid and ghosts (CFL gate paragraph of GPU
//    Implementation).
//  * Adami ghost state on the disk ring and on three lattice layers of wall
//    ghosts (eq. adami-p, eq. adami-v), body-force term (g - a_w) as in
//    Adami 2012; ring of N_g ghosts with m_g = rho0 dx 2 pi R / N_g.
//  * hard wall reflection (Channel Walls section) and a radial pull-out plus
//    reflection of the inward relative velocity for the disk.
//  * prescribed kinematics: ramp (eq. velocity-ramp) then constant
//    deceleration k v0^2, or the quadratic drag of eq. drag.
//  * two-way coupling (the extension named in the Conclusions and the
//    energy-audit discussion, kin_mode 2): after the ramp the disk moves
//    with the reaction of the ring's x force on the fluid.
//  * cell-linked list of cell size >= 2h, rebuilt at every evaluation by a
//    stable sort of the particles by cell key.
//  * the energy audit of eq. energy-audit, term by term: besides the work
//    W_boundary of the ring on the fluid, the integrals over time of the
//    fluid energy rate of every fluid-ghost pair term (W_ghost), of the
//    irreversible dissipation of the artificial and laminar viscosity
//    between fluid particles (D_av, D_visc), of the elastic energy rate of
//    the delta diffusion (W_delta), all from the midpoint rates times dt,
//    and the energy changed by the enforcement and the density clamp of the
//    corrector (W_enforce, W_clamp). What they leave of the change of the
//    fluid energy is the time-integration, XSPH and boundary-position part.
//  * the axisymmetric r-z form (axisym = 1; the first of the extensions the
//    Conclusions rank): the plane is the meridian half-plane through the
//    tank axis, x the axial coordinate, y >= 0 the radius, the sphere's
//    centre on the axis. Each fluid particle stands for a ring of fixed mass
//    M_i = 2 pi r_i(0) rho0 dx^2; its planar mass in the pair sums is
//    M_i / (2 pi r_i), so m_i / rho_i stays its area in the meridian plane.
//    The continuity equation in cylindrical coordinates adds the hoop part
//    of the divergence, -rho_i v_r,i / r_i (r_i held >= dx/2), to the
//    planar sums; the pressure gradient has no hoop part. The three ghost
//    layers below the axis are the mirror of the fluid: Shepard pressure,
//    axial velocity kept and radial velocity reversed; those inside the
//    sphere are off (zero mass). Mass, momentum, energies and the ring's
//    force are the 3D values (each particle weighted by its ring mass).
// Ghost state and rates are re-evaluated at both evaluations of a step
// (operator split of the Pipeline Provenance section).

#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Dual numbers with N tangent directions (forward-mode derivative).
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0) { for (int k = 0; k < N; ++k) d[k] = 0; }
  Dual(double x) : v(x) { for (int k = 0; k < N; ++k) d[k] = 0; }  // NOLINT
};
template <int N> Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v + b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v - b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a) { Dual<N> r; r.v = -a.v; for (int k = 0; k < N; ++k) r.d[k] = -a.d[k]; return r; }
template <int N> Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v * b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
template <int N> Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v / b.v; for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v); return r; }
template <int N> Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> Dual<N> operator*(const Dual<N>& a, double b) { Dual<N> r; r.v = a.v * b; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b; return r; }
template <int N> Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }
template <int N> Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) { a = a - b; return a; }
template <int N> Dual<N> sqrt(const Dual<N>& a) { Dual<N> r; r.v = std::sqrt(a.v); for (int k = 0; k < N; ++k) r.d[k] = a.d[k] / (2.0 * r.v); return r; }
template <int N> Dual<N> pow(const Dual<N>& a, double e) { Dual<N> r; r.v = std::pow(a.v, e); double g = e * std::pow(a.v, e - 1.0); for (int k = 0; k < N; ++k) r.d[k] = g * a.d[k]; return r; }

inline double val(double x) { return x; }
template <int N> double val(const Dual<N>& x) { return x.v; }
using std::pow;
using std::sqrt;

// ---------------------------------------------------------------------------
// Geometry and constants derived from the parameters.
struct Geom {
  double dx, h, dc, x_lo, y_lo;
  int nx, ny, ncx, ncy;
  double sigma;  // Wendland C2 2D normalisation 7 / (4 pi h^2)
  double fgrad;  // gradient factor 35 / (4 pi h^4)
  int cubic;     // 1: the cubic B-spline of eq. cubic-kernel instead
  double sigma_c;  // its 2D normalisation 10 / (7 pi h^2)
  double m_fluid, m_wall, m_disk, nu0;
};

template <class T>
void kernel_WF(const T& q, const Geom& g, T& W, T& F);

Geom make_geom(const orc_params& p) {
  Geom g;
  g.dx = p.dx;
  g.h = p.h_over_dx * p.dx;
  g.dc = p.cell_size > 0 ? p.cell_size : 2.0 * g.h;
  g.x_lo = -p.ghost_layers * p.dx;
  g.y_lo = -p.ghost_layers * p.dx;
  g.nx = (int)std::lround(p.L / p.dx);
  g.ny = (int)std::lround(p.W / p.dx);
  g.ncx = (int)std::ceil((p.L + 2.0 * p.ghost_layers * p.dx) / g.dc);
  g.ncy = (int)std::ceil((p.W + 2.0 * p.ghost_layers * p.dx) / g.dc);
  g.sigma = 7.0 / (4.0 * M_PI * g.h * g.h);
  g.fgrad = 35.0 / (4.0 * M_PI * g.h * g.h * g.h * g.h);
  g.cubic = p.kernel_type == 1;
  g.sigma_c = 10.0 / (7.0 * M_PI * g.h * g.h);
  g.m_fluid = p.rho0 * p.dx * p.dx;
  if (p.scheme == 1) {
    // summation density (Density Summation): the mass that makes the kernel
    // sum of the undisturbed square lattice equal rho0
    double S = 0.0;
    for (int j = -4; j <= 4; ++j)
      for (int i = -4; i <= 4; ++i) {
        const double q = std::sqrt((double)(i * i + j * j)) * p.dx / g.h;
        if (q >= 2.0) continue;
        double W, F;
        kernel_WF(q, g, W, F);
        S += W;
      }
    g.m_fluid = p.rho0 / S;
  }
  g.m_wall = g.m_fluid;
  // the ring: one particle layer of the fluid's areal mass density per unit arc length
  g.m_disk = p.n_disk_ghosts > 0 ? g.m_fluid / p.dx * 2.0 * M_PI * p.disk_R / p.n_disk_ghosts : 0.0;
  g.nu0 = p.mu_dyn / p.rho0;
  return g;
}

int cell_coord(double x, double lo, double dc, int n) {
  int c = (int)std::floor((x - lo) / dc);
  return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

// Wendland C2 in 2D: W = sigma (1 - q/2)^4 (2q + 1) for q < 2; grad_i W = F r_ij
// with F = -(35 / (4 pi h^4)) (1 - q/2)^3 (derivative of W divided by r).
template <class T>
void kernel_WF(const T& q, const Geom& g, T& W, T& F) {
  if (g.cubic) {
    // cubic B-spline (eq. cubic-kernel): w(q) = 1 - 3/2 q^2 + 3/4 q^3 on
    // [0, 1], (2 - q)^3 / 4 on (1, 2]; F = (1/r) dW/dr = w'(q) / (h r)
    const double h2 = g.h * g.h;
    if (val(q) <= 1.0) {
      W = g.sigma_c * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
      F = g.sigma_c * (-3.0 + 2.25 * q) / h2;
    } else {
      T s = 2.0 - q;
      W = g.sigma_c * 0.25 * s * s * s;
      F = -0.75 * g.sigma_c * s * s / (h2 * q);
    }
    return;
  }
  T s = 1.0 - 0.5 * q;
  T s2 = s * s;
  W = g.sigma * s2 * s2 * (2.0 * q + 1.0);
  F = -g.fgrad * s2 * s;
}

// Coefficients that the tangent build differentiates (alpha, delta, c0) and
// the ones that follow from them.
template <class T>
struct Coef {
  T alpha, delta, c0, B;
};

// Mie-Grueneisen law of eq. eos (eos_type 1) with the specific internal
// energy held at zero: no energy equation is evolved, so the
// (gamma0 + a mu) rho e term drops out and p depends on rho alone. With
// mu = rho/rho0 - 1 capped at mg_mu_max and C = c0:
//   compression (mu >= 0): p = rho0 C^2 mu [1 + (1 - gamma0/2) mu] / [1 - (S1 - 1) mu]^2,
//   tension (mu < 0):      p = rho0 C^2 mu.
//
// Scheme 1 evolves the specific internal energy e and adds the energy term
// of eq. eos, (gamma0 + a mu) rho e in compression and gamma0 rho e in
// tension, with rho = rho0 (1 + mu) at the same capped mu.
template <class T>
T mg_p(const T& rho, const orc_params& p, const Coef<T>& k, const T& e) {
  T mu = rho / p.rho0 - 1.0;
  if (val(mu) > p.mg_mu_max) mu = T(p.mg_mu_max);
  const T K = p.rho0 * (k.c0 * k.c0);
  const T rh = p.rho0 * (1.0 + mu);
  if (val(mu) < 0.0) return K * mu + p.mg_gamma0 * rh * e;
  const T den = 1.0 - (p.mg_s1 - 1.0) * mu;
  return K * mu * (1.0 + (1.0 - 0.5 * p.mg_gamma0) * mu) / (den * den) + (p.mg_gamma0 + p.mg_a * mu) * rh * e;
}
// Its sound speed, c^2 = dp/drho of the same law (taken at the capped mu):
// C^2 [1 + (2 - gamma0 + S1 - 1) mu] / [1 - (S1 - 1) mu]^3 in compression, C^2 in tension.
template <class T>
T mg_c(const T& rho, const orc_params& p, const Coef<T>& k) {
  T mu = rho / p.rho0 - 1.0;
  if (val(mu) > p.mg_mu_max) mu = T(p.mg_mu_max);
  if (val(mu) < 0.0) return k.c0;
  const double b = p.mg_s1 - 1.0;
  const T den = 1.0 - b * mu;
  return k.c0 * sqrt((1.0 + (2.0 - p.mg_gamma0 + b) * mu) / (den * den * den));
}
// The density at pressure q of the same law (ghost_rho_mode 1, the
// hydrostatic start): the tension branch inverted, or in compression the
// root in [0, 1/(S1 - 1)) of q (1 - b mu)^2 = K mu (1 + k1 mu), i.e. of
// (q b^2 - K k1) mu^2 - (2 q b + K) mu + q = 0, written as 2q / (B + sqrt(B^2 - 4Aq));
// capped at mg_mu_max.
template <class T>
T mg_rho(const T& q, const orc_params& p, const Coef<T>& k) {
  const T K = p.rho0 * (k.c0 * k.c0);
  if (val(q) < 0.0) return p.rho0 * (1.0 + q / K);
  const double b = p.mg_s1 - 1.0, k1 = 1.0 - 0.5 * p.mg_gamma0;
  const T A = q * (b * b) - K * k1, Bq = 2.0 * b * q + K;
  T mu = 2.0 * q / (Bq + sqrt(Bq * Bq - 4.0 * A * q));
  if (val(mu) > p.mg_mu_max) mu = T(p.mg_mu_max);
  return p.rho0 * (1.0 + mu);
}

// EOS with the cavitation cutoff p >= p_cav: Tait (eos_type 0),
// p = B((rho/rho0)^gamma - 1), c = c0 (rho/rho0)^((gamma-1)/2), or the
// Mie-Grueneisen law above.
// (e: the specific internal energy, zero except in scheme 1; the Tait law
// does not depend on it)
template <class T>
T eos_p_uncut(const T& rho, const orc_params& p, const Coef<T>& k, const T& e = T(0.0)) {
  if (p.eos_type == 1) return mg_p(rho, p, k, e);
  return k.B * (pow(rho / p.rho0, p.gamma) - 1.0);
}
template <class T>
T eos_p(const T& rho, const orc_params& p, const Coef<T>& k, const T& e = T(0.0)) {
  T pr = eos_p_uncut(rho, p, k, e);
  return val(pr) < p.p_cav ? T(p.p_cav) : pr;
}
template <class T>
T eos_c(const T& rho, const orc_params& p, const Coef<T>& k) {
  if (p.eos_type == 1) return mg_c(rho, p, k);
  return k.c0 * pow(rho / p.rho0, 0.5 * (p.gamma - 1.0));
}
// inverse of the EOS for a pressure q >= p_cav (no cutoff branch)
template <class T>
T eos_rho(const T& q, const orc_params& p, const Coef<T>& k) {
  if (p.eos_type == 1) return mg_rho(q, p, k);
  return p.rho0 * pow(1.0 + q / k.B, 1.0 / p.gamma);
}

// A particle as seen by the pair law.
template <class T>
struct PV {
  T x, y, vx, vy, rho, P, c;  // P = p / rho^2
  double m;
  int kind;  // 0 fluid, 1 wall ghost, 2 disk ghost
};

template <class T>
struct Acc {
  T D, ax, ay, Vx, Vy, fdx;
  T E;  // scheme 1: rate of the specific internal energy (artificial-viscosity heating)
  // energy audit, per unit mass of particle a (values only)
  double av, visc, del, ghost;
  Acc() : D(0.0), ax(0.0), ay(0.0), Vx(0.0), Vy(0.0), fdx(0.0), E(0.0), av(0), visc(0), del(0), ghost(0) {}
};

// Contribution of neighbour b to the rates of fluid particle a.
template <class T>
void pair_law(const PV<T>& a, const PV<T>& b, const orc_params& p, const Geom& g,
              const Coef<T>& k, Acc<T>& acc) {
  T rx = a.x - b.x, ry = a.y - b.y;
  T r2 = rx * rx + ry * ry;
  if (!(val(r2) < 4.0 * g.h * g.h)) return;
  T r = sqrt(r2);
  T q = r / g.h;
  T W, F;
  kernel_WF(q, g, W, F);
  T vxij = a.vx - b.vx, vyij = a.vy - b.vy;
  T vr = vxij * rx + vyij * ry;
  T rbar = 0.5 * (a.rho + b.rho);
  T cbar = 0.5 * (a.c + b.c);
  T denom = r2 + p.eta2 * g.h * g.h;
  T Pi(0.0);
  if (val(vr) < 0.0) {
    T mu = g.h * vr / denom;
    Pi = -1.0 * k.alpha * cbar * mu / rbar;
    // quadratic (von Neumann-Richtmyer) term of the Monaghan form, which the
    // paper leaves out at its Mach numbers and names for faster impacts
    Pi = Pi + p.beta * mu * mu / rbar;
  }
  // continuity: d rho_i/dt = sum_j m_j v_ij . grad_i W_ij
  acc.D += b.m * vr * F;
  // delta diffusion (fluid pairs): delta h c0 sum_j V_j psi_ij . grad_i W_ij,
  // psi_ij = 2 (rho_j - rho_i) (r_j - r_i) / |r_ij|^2
  T dd(0.0);
  if (b.kind == 0) dd = 2.0 * k.delta * g.h * k.c0 * (b.m / b.rho) * (a.rho - b.rho) * F;
  acc.D += dd;
  // pressure + artificial viscosity, symmetric form
  T s = a.P + b.P + Pi;
  acc.ax -= b.m * s * F * rx;
  acc.ay -= b.m * s * F * ry;
  if (b.kind == 2) acc.fdx -= b.m * s * F * rx;
  // internal energy (scheme 1): half of the pair's artificial-viscosity
  // dissipation, (1/2) m_j Pi_ij v_ij . grad_i W_ij >= 0, over every neighbour
  acc.E += 0.5 * b.m * Pi * F * vr;
  // laminar viscosity (Lo-Shao): sum_j 4 nu0 m_j (r_ij . grad W) / ((rho_i + rho_j)(r^2 + eta^2 h^2)) v_ij
  T lam = b.m * 4.0 * g.nu0 * F * r2 / ((a.rho + b.rho) * denom);
  acc.ax += lam * vxij;
  acc.ay += lam * vyij;
  // energy audit. Between fluid particles the pressure work cancels the
  // elastic energy rate of the continuity term pair by pair; what is left is
  // the dissipation of the viscous terms, half to each particle of the pair:
  // (1/2) m_j Pi_ij F v_ij.r_ij >= 0 and -(1/2) lam |v_ij|^2 >= 0 (F < 0),
  // and the delta term's elastic energy rate P_i dd. A ghost pair is counted
  // whole: the work of its pressure, AV and laminar forces on v_i plus the
  // elastic energy rate P_i m_g F v_ig.r_ig of its continuity term.
  if (b.kind == 0) {
    acc.av += 0.5 * val(b.m * Pi * F * vr);
    acc.visc -= 0.5 * val(lam * (vxij * vxij + vyij * vyij));
    acc.del += val(a.P * dd);
  } else {
    acc.ghost += val(-b.m * s * F * (rx * a.vx + ry * a.vy) + lam * (vxij * a.vx + vyij * a.vy) +
                     a.P * b.m * vr * F);
  }
  // XSPH over fluid neighbours
  if (b.kind == 0) {
    T w = p.eps_xsph * (b.m / rbar) * W;
    acc.Vx += w * (b.vx - a.vx);
    acc.Vy += w * (b.vy - a.vy);
  }
}

// Prescribed disk kinematics (centre x, velocity, acceleration along +x).
void kinematics(int mode, double v0, double t_ramp, double coef, double x0, double t, double* xo,
                double* vo, double* ao) {
  if (t < t_ramp) {
    *vo = v0 * t / t_ramp;
    *ao = v0 / t_ramp;
    *xo = x0 + 0.5 * v0 * t * t / t_ramp;
    return;
  }
  double tau = t - t_ramp;
  double xr = x0 + 0.5 * v0 * t_ramp;
  if (mode == 2) {  // two-way coupling: this prescribed law only until the first coupled step
    *vo = v0;
    *ao = 0;
    *xo = xr + v0 * tau;
    return;
  }
  if (mode == 1) {  // quadratic drag dv/dt = -k v^2
    double k = coef;
    double v = v0 / (1.0 + k * v0 * tau);
    *vo = v;
    *ao = -k * v * v;
    *xo = k > 0 ? xr + std::log1p(k * v0 * tau) / k : xr + v0 * tau;
    return;
  }
  double ad = coef;  // constant deceleration, stops at v = 0
  if (ad > 0 && tau >= v0 / ad) {
    *vo = 0;
    *ao = 0;
    *xo = xr + 0.5 * v0 * v0 / ad;
    return;
  }
  *vo = v0 - ad * tau;
  *ao = -ad;
  *xo = xr + v0 * tau - 0.5 * ad * tau * tau;
}

// ---------------------------------------------------------------------------
// Tabulated prescribed motion (kin_mode 3): rows (t, x, v, a) with t
// strictly increasing, x the absolute centre position. Between two rows each
// column is interpolated linearly in t (a row's own time gives the row);
// before the first row and after the last the centre moves on at that row's
// velocity with zero acceleration.
void table_kinematics(const std::vector<double>& tab, double t, double* xo, double* vo, double* ao) {
  const int n = (int)(tab.size() / 4);
  if (n == 0) {
    *xo = *vo = *ao = 0.0;
    return;
  }
  if (t < tab[0] || n == 1) {
    const int r = t < tab[0] ? 0 : n - 1;
    *xo = tab[4 * r + 1] + tab[4 * r + 2] * (t - tab[4 * r]);
    *vo = tab[4 * r + 2];
    *ao = 0.0;
    return;
  }
  // the last row with t_k <= t
  std::vector<double> ts(n);
  for (int k = 0; k < n; ++k) ts[k] = tab[4 * k];
  const int k = (int)(std::upper_bound(ts.begin(), ts.end(), t) - ts.begin()) - 1;
  if (k >= n - 1) {  // at or past the last row
    const double* r = &tab[4 * (n - 1)];
    *xo = t == r[0] ? r[1] : r[1] + r[2] * (t - r[0]);
    *vo = r[2];
    *ao = t == r[0] ? r[3] : 0.0;
    return;
  }
  const double w = (t - tab[4 * k]) / (tab[4 * (k + 1)] - tab[4 * k]);
  *xo = tab[4 * k + 1] + w * (tab[4 * (k + 1) + 1] - tab[4 * k + 1]);
  *vo = tab[4 * k + 2] + w * (tab[4 * (k + 1) + 2] - tab[4 * k + 2]);
  *ao = tab[4 * k + 3] + w * (tab[4 * (k + 1) + 3] - tab[4 * k + 3]);
}

template <class T>
struct Sim {
  orc_params P;
  Geom G;
  Coef<T> K;
  int Nf = 0, Nw = 0, Nd = 0;
  // fluid state by fluid id (scheme 1: v at the half step, rho the last
  // summed density, e the specific internal energy)
  std::vector<T> x, y, vx, vy, rho, e;
  double dt_prev = 0.0;  // scheme 1: dt of the previous step (0 before the first)
  // axisymmetric form: ring mass per radian M_i / (2 pi) = r_i(0) rho0 dx^2 by fluid id
  std::vector<double> mring;
  // ghosts by ghost index: walls first, then the disk ring; goff: a ghost
  // below the axis inside the sphere, off for the current evaluation
  std::vector<double> gx, gy, gm;
  std::vector<char> goff;
  std::vector<T> gp, grho, gvx, gvy;
  // cell list: storage order (global ids) and cell ranges
  std::vector<int> order, cell_start, key;
  double t = 0.0;
  long step = 0;
  std::vector<double> dt_table;
  std::vector<double> probe_rows;  // per row: t, dt, then probes
  std::vector<T> probe_vals;
  std::vector<double> diag_rows;
  T J = T(0.0);
  double w_boundary = 0.0;
  long n_clamp = 0, n_enforce = 0;
  // energy audit integrals: D_av, D_visc, W_delta, W_ghost, W_enforce, W_clamp
  double audit[6] = {0, 0, 0, 0, 0, 0};
  mutable double audit_rate[4] = {0, 0, 0, 0};
  // disk state at the current evaluation
  double dx_c = 0, dv = 0, da = 0;
  // two-way coupling (kin_mode 2): from the first step that starts at or
  // after the ramp, the disk state at t evolves with the ring's force
  bool coupled = false;
  double xc = 0, vc = 0, ac = 0;

  int N() const { return Nf + Nw + Nd; }

  // the radius below which the hoop term and the planar mass hold it (the
  // first lattice row)
  double rmin() const { return 0.5 * P.dx; }
  // planar mass of fluid particle i in the pair sums: m_fluid, or in the
  // axisymmetric form its ring mass over 2 pi r_i
  double plan_mass(int i) const {
    if (!P.axisym) return G.m_fluid;
    return mring[i] / std::max(val(y[i]), rmin());
  }
  // its weight in the mass, momentum and energy sums and the ring force:
  // m_fluid (per unit depth), or the ring mass 2 pi M_i / (2 pi)
  double weight3(int i) const { return P.axisym ? 2.0 * M_PI * mring[i] : G.m_fluid; }

  void setup(const orc_params& p, int n_init, const double* init) {
    P = p;
    G = make_geom(p);
    // fluid (S1): lattice points ((i+1/2)dx, (j+1/2)dx), id = j nx + i, disk interior removed
    if (init == nullptr) {
      const double cx = p.disk_x0, cy = p.disk_y0, R = p.disk_R;
      for (int j = 0; j < G.ny; ++j)
        for (int i = 0; i < G.nx; ++i) {
          double xx = (i + 0.5) * p.dx, yy = (j + 0.5) * p.dx;
          if (R > 0 && (xx - cx) * (xx - cx) + (yy - cy) * (yy - cy) < R * R) continue;
          double r0 = p.rho0;
          if (p.init_mode == 1) {  // hydrostatic: the EOS inverse of rho0 |g| (W - y)
            Coef<double> k;
            k.c0 = p.c0; k.B = p.rho0 * p.c0 * p.c0 / p.gamma;
            r0 = eos_rho(p.rho0 * std::fabs(p.gravity_y) * (p.W - yy), p, k);
          }
          x.push_back(xx); y.push_back(yy); vx.push_back(0.0); vy.push_back(0.0); rho.push_back(r0);
        }
    } else {
      for (int k = 0; k < n_init; ++k) {
        x.push_back(init[5 * k]); y.push_back(init[5 * k + 1]);
        vx.push_back(init[5 * k + 2]); vy.push_back(init[5 * k + 3]); rho.push_back(init[5 * k + 4]);
      }
    }
    Nf = (int)x.size();
    e.assign(Nf, T(0.0));
    mring.assign(Nf, 0.0);
    if (p.axisym)
      for (int i = 0; i < Nf; ++i) mring[i] = val(y[i]) * G.m_fluid;
    // wall ghosts (S2): the lattice continued ghost_layers deep around the box, j outer
    const int Lg = p.ghost_layers;
    for (int j = -Lg; j < G.ny + Lg; ++j)
      for (int i = -Lg; i < G.nx + Lg; ++i) {
        if (i >= 0 && i < G.nx && j >= 0 && j < G.ny) continue;
        gx.push_back((i + 0.5) * p.dx); gy.push_back((j + 0.5) * p.dx); gm.push_back(G.m_wall);
      }
    Nw = (int)gx.size();
    // disk ring (S3)
    Nd = p.disk_R > 0 ? p.n_disk_ghosts : 0;
    for (int k = 0; k < Nd; ++k) { gx.push_back(0); gy.push_back(0); gm.push_back(G.m_disk); }
    goff.assign(Nw + Nd, 0);
    gp.assign(Nw + Nd, T(0.0)); grho.assign(Nw + Nd, T(p.rho0));
    gvx.assign(Nw + Nd, T(0.0)); gvy.assign(Nw + Nd, T(0.0));
    order.resize(N());
    for (int k = 0; k < N(); ++k) order[k] = k;
    key.assign(N(), 0);
    cell_start.assign(G.ncx * G.ncy + 1, 0);
    probe_vals.assign(P.n_probes, T(0.0));
    record_diag(0.0, 0.0);
  }

  void set_coef(const T& alpha, const T& delta, const T& c0) {
    K.alpha = alpha; K.delta = delta; K.c0 = c0;
    K.B = P.rho0 * c0 * c0 / P.gamma;
  }

  std::vector<double> kin_tab;  // kin_mode 3: rows (t, x, v, a)

  // the prescribed disk motion at time tt (closed forms, or the table)
  void kin(double tt, double* x_, double* v_, double* a_) const {
    if (P.kin_mode == 3 && kin_tab.empty()) { *x_ = P.disk_x0; *v_ = 0.0; *a_ = 0.0; }
    else if (P.kin_mode == 3) table_kinematics(kin_tab, tt, x_, v_, a_);
    else kinematics(P.kin_mode, P.kin_v0, P.kin_t_ramp, P.kin_coef, P.disk_x0, tt, x_, v_, a_);
  }

  // disk centre, velocity and acceleration at time tt of the current step
  // (coupled: extrapolated from the state at t with its latest acceleration)
  void disk_state(double tt) {
    if (coupled) {
      const double tau = tt - t;
      dx_c = xc + tau * vc;
      dv = vc + tau * ac;
      da = ac;
    } else {
      kin(tt, &dx_c, &dv, &da);
    }
  }

  // disk ghosts at angle 2 pi k / N_g around the centre (eq. adami-p text)
  void place_disk(double tt) {
    disk_state(tt);
    for (int k = 0; k < Nd; ++k) {
      double th = 2.0 * M_PI * k / Nd;
      gx[Nw + k] = dx_c + P.disk_R * std::cos(th);
      gy[Nw + k] = P.disk_y0 + P.disk_R * std::sin(th);
    }
  }

  double px(int id) const { return id < Nf ? val(x[id]) : gx[id - Nf]; }
  double py(int id) const { return id < Nf ? val(y[id]) : gy[id - Nf]; }

  // keys for every particle and a stable re-sort of the storage order by key
  void build_cells() {
    for (int id = 0; id < N(); ++id) {
      int cx = cell_coord(px(id), G.x_lo, G.dc, G.ncx);
      int cy = cell_coord(py(id), G.y_lo, G.dc, G.ncy);
      key[id] = cy * G.ncx + cx;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    std::fill(cell_start.begin(), cell_start.end(), 0);
    for (int id = 0; id < N(); ++id) cell_start[key[id] + 1]++;
    for (size_t k = 1; k < cell_start.size(); ++k) cell_start[k] += cell_start[k - 1];
  }

  // visit ids in the 3x3 block of cells around (xx, yy): rows bottom to top,
  // cells left to right, storage order inside a cell
  template <class Fn>
  void for_neighbours(double xx, double yy, Fn&& fn) const {
    int cx = cell_coord(xx, G.x_lo, G.dc, G.ncx);
    int cy = cell_coord(yy, G.y_lo, G.dc, G.ncy);
    for (int dy = -1; dy <= 1; ++dy) {
      int yy2 = cy + dy;
      if (yy2 < 0 || yy2 >= G.ncy) continue;
      for (int dxx = -1; dxx <= 1; ++dxx) {
        int xx2 = cx + dxx;
        if (xx2 < 0 || xx2 >= G.ncx) continue;
        int K2 = yy2 * G.ncx + xx2;
        for (int k = cell_start[K2]; k < cell_start[K2 + 1]; ++k) fn(order[k]);
      }
    }
  }

  // Shepard sums over fluid within 2h of point (xx, yy)
  void shepard(double xx, double yy, const std::vector<T>& pf, T& SW, T& Sp, T& Srx, T& Sry,
               T& Svx, T& Svy) const {
    SW = Sp = Srx = Sry = Svx = Svy = T(0.0);
    for_neighbours(xx, yy, [&](int j) {
      if (j >= Nf) return;
      T rx = xx - x[j], ry = yy - y[j];
      T r2 = rx * rx + ry * ry;
      if (!(val(r2) < 4.0 * G.h * G.h)) return;
      T W, F;
      kernel_WF(sqrt(r2) / G.h, G, W, F);
      SW += W;
      Sp += pf[j] * W;
      Srx += rho[j] * rx * W;
      Sry += rho[j] * ry * W;
      Svx += vx[j] * W;
      Svy += vy[j] * W;
    });
  }

  // Adami ghost state (eq. adami-p, eq. adami-v) for every ghost
  void ghosts(const std::vector<T>& pf) {
    const int NG = Nw + Nd;
#pragma omp parallel for schedule(static)
    for (int g = 0; g < NG; ++g) {
      double vwx = 0, awx = 0;
      if (g >= Nw) { vwx = dv; awx = da; }
      // axisymmetric form: a wall ghost below the axis mirrors the fluid, and
      // is off inside the sphere (whose centre is on the axis)
      const bool axis = P.axisym && g < Nw && gy[g] < 0.0;
      goff[g] = 0;
      if (axis && Nd > 0 &&
          (gx[g] - dx_c) * (gx[g] - dx_c) + (gy[g] - P.disk_y0) * (gy[g] - P.disk_y0) < P.disk_R * P.disk_R) {
        goff[g] = 1;
        gp[g] = T(0.0); grho[g] = T(P.rho0); gvx[g] = T(0.0); gvy[g] = T(0.0);
        continue;
      }
      T SW, Sp, Srx, Sry, Svx, Svy;
      shepard(gx[g], gy[g], pf, SW, Sp, Srx, Sry, Svx, Svy);
      T pg, vgx, vgy;
      if (val(SW) > 0.0) {
        // body-force term (g - a_w) . sum_j rho_j (r_g - r_j) W_gj
        pg = (Sp + (0.0 - awx) * Srx + (P.gravity_y - 0.0) * Sry) / SW;
        vgx = 2.0 * vwx - Svx / SW;
        vgy = 0.0 - Svy / SW;
        if (axis) vgx = Svx / SW;  // slip: the axial velocity is kept, the radial one reversed
      } else {
        pg = T(0.0);
        vgx = T(vwx);
        vgy = T(0.0);
      }
      if (val(pg) < P.p_cav) pg = T(P.p_cav);
      T rg;
      if (P.ghost_rho_mode == 0) rg = P.rho0 * (1.0 + pg / (P.rho0 * K.c0 * K.c0));  // linear branch
      else rg = eos_rho(pg, P, K);
      gp[g] = pg; grho[g] = rg; gvx[g] = vgx; gvy[g] = vgy;
    }
  }

  // particle view for the pair law
  PV<T> view(int id, const std::vector<T>& pf) const {
    PV<T> v;
    if (id < Nf) {
      v.x = x[id]; v.y = y[id]; v.vx = vx[id]; v.vy = vy[id]; v.rho = rho[id];
      v.P = pf[id] / (rho[id] * rho[id]);
      v.c = eos_c(rho[id], P, K);
      v.m = plan_mass(id); v.kind = 0;
    } else {
      int g = id - Nf;
      v.x = T(gx[g]); v.y = T(gy[g]); v.vx = gvx[g]; v.vy = gvy[g]; v.rho = grho[g];
      v.P = gp[g] / (grho[g] * grho[g]);
      v.c = eos_c(grho[g], P, K);
      v.m = goff[g] ? 0.0 : gm[g]; v.kind = g < Nw ? 1 : 2;
    }
    return v;
  }

  // rates of every fluid particle; returns the x force of the disk on the fluid
  T rates(const std::vector<T>& pf, std::vector<T>& D, std::vector<T>& ax, std::vector<T>& ay,
          std::vector<T>& Vx, std::vector<T>& Vy) const {
    std::vector<T> fdx(Nf);
    std::vector<double> au(4 * (size_t)Nf);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < Nf; ++i) {
      PV<T> a = view(i, pf);
      Acc<T> acc;
      for_neighbours(val(x[i]), val(y[i]), [&](int j) {
        if (j == i) return;
        pair_law(a, view(j, pf), P, G, K, acc);
      });
      D[i] = P.scheme == 1 ? acc.E : acc.D;
      // axisymmetric form: the hoop part of the divergence, -rho v_r / r
      if (P.axisym) D[i] = D[i] - rho[i] * vy[i] / std::max(val(y[i]), rmin());
      ax[i] = acc.ax;
      ay[i] = acc.ay + P.gravity_y;
      Vx[i] = vx[i] + acc.Vx;
      Vy[i] = vy[i] + acc.Vy;
      fdx[i] = weight3(i) * acc.fdx;
      au[4 * (size_t)i] = acc.av;
      au[4 * (size_t)i + 1] = acc.visc;
      au[4 * (size_t)i + 2] = acc.del;
      au[4 * (size_t)i + 3] = acc.ghost;
    }
    T f(0.0);
    for (int i = 0; i < Nf; ++i) f += fdx[i];
    for (int q = 0; q < 4; ++q) {
      double z = 0.0;
      for (int i = 0; i < Nf; ++i) z += weight3(i) * au[4 * (size_t)i + q];
      audit_rate[q] = z;
    }
    return f;
  }

  void fluid_pressure(std::vector<T>& pf) const {
    pf.resize(Nf);
    for (int i = 0; i < Nf; ++i) pf[i] = eos_p(rho[i], P, K, e[i]);
  }

  // Summation density (eq. density-sum) of every fluid particle over the fluid
  // and ghosts in support, itself included, clamped to [rho_lo, rho_hi] rho0
  void sum_density() {
    const double lo = P.rho_lo * P.rho0, hi = P.rho_hi * P.rho0;
    long nc = 0;
#pragma omp parallel for schedule(static) reduction(+ : nc)
    for (int i = 0; i < Nf; ++i) {
      T sum(0.0);
      for_neighbours(val(x[i]), val(y[i]), [&](int j) {
        if (j == i) {  // the particle itself, at r = 0
          T W0, F0;
          kernel_WF(T(0.0), G, W0, F0);
          sum += G.m_fluid * W0;
          return;
        }
        T rx = j < Nf ? x[i] - x[j] : x[i] - gx[j - Nf];
        T ry = j < Nf ? y[i] - y[j] : y[i] - gy[j - Nf];
        T r2 = rx * rx + ry * ry;
        if (!(val(r2) < 4.0 * G.h * G.h)) return;
        T W, F;
        kernel_WF(sqrt(r2) / G.h, G, W, F);
        sum += (j < Nf ? G.m_fluid : gm[j - Nf]) * W;
      });
      if (val(sum) < lo) { sum = T(lo); nc++; }
      if (val(sum) > hi) { sum = T(hi); nc++; }
      rho[i] = sum;
    }
    n_clamp += nc;
  }

  // hard walls (Channel Walls section) then the disk: radial pull-out to
  // R + eps and reflection of the inward normal velocity relative to the disk
  bool enforce(T& xx, T& yy, T& ux, T& uy, double cx, double cy, double vd) const {
    bool hit = false;
    const double e = P.eps_wall;
    if (val(xx) < e) { xx = T(e); ux = -1.0 * ux; hit = true; }
    if (val(xx) > P.L - e) { xx = T(P.L - e); ux = -1.0 * ux; hit = true; }
    if (val(yy) < e) { yy = T(e); uy = -1.0 * uy; hit = true; }
    if (val(yy) > P.W - e) { yy = T(P.W - e); uy = -1.0 * uy; hit = true; }
    if (Nd > 0) {
      T rx = xx - cx, ry = yy - cy;
      T d2 = rx * rx + ry * ry;
      if (val(d2) < P.disk_R * P.disk_R) {
        T nx(-1.0), ny(0.0);
        if (val(d2) > 0.0) { T d = sqrt(d2); nx = rx / d; ny = ry / d; }
        xx = cx + (P.disk_R + e) * nx;
        yy = cy + (P.disk_R + e) * ny;
        T w = (ux - vd) * nx + uy * ny;
        if (val(w) < 0.0) { ux = ux - 2.0 * w * nx; uy = uy - 2.0 * w * ny; }
        hit = true;
      }
    }
    return hit;
  }

  // phi = clamp(phi0 + h D), v = v0 + h a, r = r0 + h V, then enforcement
  // against the disk at centre x cx, velocity vd
  void advance(const std::vector<T>& x0, const std::vector<T>& y0, const std::vector<T>& vx0,
               const std::vector<T>& vy0, const std::vector<T>& rho0, double hdt,
               const std::vector<T>& D, const std::vector<T>& ax, const std::vector<T>& ay,
               const std::vector<T>& Vx, const std::vector<T>& Vy, double cx, double vd,
               bool corrector) {
    const double lo = P.rho_lo * P.rho0, hi = P.rho_hi * P.rho0;
    for (int i = 0; i < Nf; ++i) {
      T r = rho0[i] + hdt * D[i];
      const double r_free = val(r);
      if (val(r) < lo) { r = T(lo); n_clamp++; }
      if (val(r) > hi) { r = T(hi); n_clamp++; }
      // energy the clamp and the enforcement of the new state add (corrector)
      if (corrector && val(r) != r_free) audit[5] += weight3(i) * (e_el(val(r)) - e_el(r_free));
      T ux = vx0[i] + hdt * ax[i], uy = vy0[i] + hdt * ay[i];
      T xx = x0[i] + hdt * Vx[i], yy = y0[i] + hdt * Vy[i];
      const double k_free = val(ux) * val(ux) + val(uy) * val(uy);
      if (enforce(xx, yy, ux, uy, cx, P.disk_y0, vd)) {
        n_enforce++;
        if (corrector) audit[4] += 0.5 * weight3(i) * (val(ux) * val(ux) + val(uy) * val(uy) - k_free);
      }
      x[i] = xx; y[i] = yy; vx[i] = ux; vy[i] = uy; rho[i] = r;
    }
  }

  // Shepard average of fluid pressure at the probe points
  void probes(const std::vector<T>& pf) {
    for (int k = 0; k < P.n_probes; ++k) {
      T SW, Sp, a, b, c, d;
      shepard(P.probe_xy[2 * k], P.probe_xy[2 * k + 1], pf, SW, Sp, a, b, c, d);
      probe_vals[k] = val(SW) > 0.0 ? Sp / SW : T(0.0);
    }
  }

  double vmax_now() const {
    double m = 0.0;
    for (int i = 0; i < Nf; ++i) m = std::max(m, std::hypot(val(vx[i]), val(vy[i])));
    for (int g = 0; g < Nw + Nd; ++g) m = std::max(m, std::hypot(val(gvx[g]), val(gvy[g])));
    return m;
  }

  // one evaluation at time te on the current fluid state: disk placement,
  // cell list, ghost state
  void prepare(double te, std::vector<T>& pf) {
    place_disk(te);
    build_cells();
    if (P.scheme == 1) sum_density();
    fluid_pressure(pf);
    ghosts(pf);
  }

  // Scheme 1 (the paper as published), one evaluation per step at state n
  // (positions r^n, half-step velocities v^(n-1/2), internal energy e^n):
  // the summed and clamped density with the energy term of the EOS, the
  // ghosts, probes and CFL step at t^n, then the merged leapfrog kick
  // v^(n+1/2) = v^(n-1/2) + (dt^(n-1) + dt^n)/2 a^n (velocity-Stormer-Verlet
  // with a variable step; dt^(-1) = 0 starts it with a half kick), the drift
  // r^(n+1) = r^n + dt^n (v^(n+1/2) + the XSPH correction of eq. xsph),
  // e^(n+1) = e^n + dt^n de/dt^n, and the wall and disk enforcement at t^(n+1).
  void one_step_leapfrog() {
    std::vector<T> pf, D(Nf), ax(Nf), ay(Nf), Vx(Nf), Vy(Nf);
    prepare(t, pf);
    probes(pf);
    const double vmax = vmax_now();
    const double dt = (step < (long)dt_table.size()) ? dt_table[step] : P.cfl * G.h / (val(K.c0) + vmax);
    probe_rows.push_back(t);
    probe_rows.push_back(dt);
    for (int k = 0; k < P.n_probes; ++k) {
      probe_rows.push_back(val(probe_vals[k]));
      J += probe_vals[k] * dt;
    }
    const T fdx = rates(pf, D, ax, ay, Vx, Vy);
    w_boundary += dt * val(fdx) * dv;
    double x1, v1, a1;
    kin(t + dt, &x1, &v1, &a1);
    const double kick = 0.5 * (dt_prev + dt);
    for (int i = 0; i < Nf; ++i) {
      T ux = vx[i] + kick * ax[i], uy = vy[i] + kick * ay[i];
      T xx = x[i] + dt * (ux + (Vx[i] - vx[i])), yy = y[i] + dt * (uy + (Vy[i] - vy[i]));
      e[i] = e[i] + dt * D[i];
      if (enforce(xx, yy, ux, uy, x1, P.disk_y0, v1)) n_enforce++;
      x[i] = xx; y[i] = yy; vx[i] = ux; vy[i] = uy;
    }
    dt_prev = dt;
    t += dt;
    step++;
    if (P.diag_every > 0 && step % P.diag_every == 0) record_diag(dt, vmax);
  }

  void one_step() {
    if (P.scheme == 1) {
      one_step_leapfrog();
      return;
    }
    std::vector<T> pf, D(Nf), ax(Nf), ay(Nf), Vx(Nf), Vy(Nf);
    const std::vector<T> x0 = x, y0 = y, vx0 = vx, vy0 = vy, rho0 = rho;
    if (P.kin_mode == 2 && !coupled && t >= P.kin_t_ramp) {
      // the first step at or after the ramp starts from the prescribed state
      kinematics(P.kin_mode, P.kin_v0, P.kin_t_ramp, P.kin_coef, P.disk_x0, t, &xc, &vc, &ac);
      coupled = true;
    }
    // evaluation at state n
    prepare(t, pf);
    probes(pf);
    double vmax = vmax_now();
    double dt = (step < (long)dt_table.size()) ? dt_table[step]
                                               : P.cfl * G.h / (val(K.c0) + vmax);
    probe_rows.push_back(t);
    probe_rows.push_back(dt);
    for (int k = 0; k < P.n_probes; ++k) {
      probe_rows.push_back(val(probe_vals[k]));
      J += probe_vals[k] * dt;
    }
    rates(pf, D, ax, ay, Vx, Vy);
    // predictor to t + dt/2
    disk_state(t + 0.5 * dt);
    advance(x0, y0, vx0, vy0, rho0, 0.5 * dt, D, ax, ay, Vx, Vy, dx_c, dv, false);
    // evaluation at the midpoint state
    prepare(t + 0.5 * dt, pf);
    T fdx = rates(pf, D, ax, ay, Vx, Vy);
    for (int q = 0; q < 4; ++q) audit[q] += dt * audit_rate[q];
    double x1, v1, a1 = 0.0;
    if (coupled) {
      // the disk takes the reaction -f of the ring's force f on the fluid:
      // M dv/dt = -f with f at t + dt/2, trapezoidal position; the boundary
      // work uses the mean velocity of the step, so that it equals the
      // disk's kinetic energy loss
      a1 = -val(fdx) / P.disk_mass;
      v1 = vc + dt * a1;
      x1 = xc + dt * 0.5 * (vc + v1);
      w_boundary += dt * val(fdx) * (0.5 * (vc + v1));
    } else {
      w_boundary += dt * val(fdx) * dv;
      double a_;
      kin(t + dt, &x1, &v1, &a_);
    }
    // corrector from state n with the midpoint rates
    advance(x0, y0, vx0, vy0, rho0, dt, D, ax, ay, Vx, Vy, x1, v1, true);
    if (coupled) {
      xc = x1;
      vc = v1;
      ac = a1;
    }
    t += dt;
    step++;
    if (P.diag_every > 0 && step % P.diag_every == 0) record_diag(dt, vmax);
  }

  // the disk state at t
  void current_disk(double* x_, double* v_, double* a_) const {
    if (coupled) {
      *x_ = xc;
      *v_ = vc;
      *a_ = ac;
    } else {
      kin(t, x_, v_, a_);
    }
  }

  // specific elastic energy int_{rho0}^{r} p / rho^2 drho of the EOS with its
  // cutoff branch: closed form for Tait; for the Mie-Grueneisen law, per unit
  // mu = rho/rho0 - 1 the integrand is p / (rho0 (1 + mu)^2), summed by the
  // composite Simpson rule over each of its smooth pieces (breaks at the
  // cutoff and at the compression cap)
  double e_el(double r) const {
    if (P.eos_type == 1) {
      Coef<double> k;
      k.c0 = val(K.c0); k.B = val(K.B);
      auto f = [&](double m) { return eos_p(P.rho0 * (1.0 + m), P, k) / (P.rho0 * (1.0 + m) * (1.0 + m)); };
      auto simpson = [&](double a, double b) {
        const int n = 256;
        double sum = f(a) + f(b);
        for (int i = 1; i < n; ++i) sum += (i % 2 ? 4.0 : 2.0) * f(a + (b - a) * i / n);
        return sum * (b - a) / (3.0 * n);
      };
      const double mu = r / P.rho0 - 1.0;
      const double mu_cav = P.p_cav / (P.rho0 * k.c0 * k.c0);
      const double brk = mu < 0.0 ? std::max(mu, mu_cav) : std::min(mu, P.mg_mu_max);
      return simpson(0.0, brk) + simpson(brk, mu);
    }
    const double g = P.gamma, r0 = P.rho0, B = val(K.B);
    auto e_tait = [&](double q) {
      return B * ((std::pow(q, g - 1.0) - std::pow(r0, g - 1.0)) / ((g - 1.0) * std::pow(r0, g)) +
                  1.0 / q - 1.0 / r0);
    };
    double rc = r0 * std::pow(1.0 + P.p_cav / B, 1.0 / g);
    if (r >= rc) return e_tait(r);
    return e_tait(rc) + P.p_cav * (1.0 / rc - 1.0 / r);
  }

  void record_diag(double dt, double vmax) {
    double M = 0, px_ = 0, py_ = 0, ke = 0, eel = 0, epot = 0, eth = 0;
    long ncav = 0;
    for (int i = 0; i < Nf; ++i) {
      double m = weight3(i), u = val(vx[i]), w = val(vy[i]), r = val(rho[i]);
      M += m;
      px_ += m * u;
      py_ += m * w;
      ke += 0.5 * m * (u * u + w * w);
      epot += m * (-P.gravity_y) * val(y[i]);
      eel += m * e_el(r);
      eth += m * val(e[i]);
      if (val(eos_p_uncut(T(r), P, K, e[i])) <= P.p_cav) ncav++;
    }
    double xd, vd, ad;
    current_disk(&xd, &vd, &ad);
    double row[ORC_NDIAG] = {t, dt, vmax, M, px_, py_, ke, eel, epot, 0.5 * P.disk_mass * vd * vd,
                             w_boundary, (double)step, (double)n_clamp, (double)ncav,
                             (double)n_enforce, audit[0], audit[1], audit[2], audit[3], audit[4],
                             audit[5], eth};
    diag_rows.insert(diag_rows.end(), row, row + ORC_NDIAG);
  }
};

using SimD = Sim<double>;

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

void* orc_create(const orc_params* p, int n_init, const double* init) {
  if (p->scheme == 1 && p->kin_mode == 2) return nullptr;  // the coupled disk is not built for scheme 1
  // the axisymmetric form: scheme 0, no gravity across the axis
  if (p->axisym && (p->scheme != 0 || p->gravity_y != 0.0)) return nullptr;
  SimD* s = new SimD();
  s->P = *p;
  s->set_coef(p->alpha, p->delta, p->c0);
  s->setup(*p, n_init, init);
  return s;
}
void orc_destroy(void* s) { delete static_cast<SimD*>(s); }
int orc_num_fluid(void* s) { return static_cast<SimD*>(s)->Nf; }
int orc_num_ghost(void* s) { auto* q = static_cast<SimD*>(s); return q->Nw + q->Nd; }
int orc_num_cells(void* s) { auto* q = static_cast<SimD*>(s); return q->G.ncx * q->G.ncy; }
void orc_set_dt_table(void* s, int n, const double* dt) {
  static_cast<SimD*>(s)->dt_table.assign(dt, dt + (n > 0 ? n : 0));
}
int orc_step(void* s, int n) {
  auto* q = static_cast<SimD*>(s);
  for (int k = 0; k < n; ++k) q->one_step();
  return 0;
}
void orc_get_fluid(void* s, double* t, double* x, double* y, double* vx, double* vy, double* rho) {
  auto* q = static_cast<SimD*>(s);
  if (t) *t = q->t;
  for (int i = 0; i < q->Nf; ++i) {
    x[i] = q->x[i]; y[i] = q->y[i]; vx[i] = q->vx[i]; vy[i] = q->vy[i]; rho[i] = q->rho[i];
  }
}
void orc_set_fluid(void* s, double t, const double* x, const double* y, const double* vx,
                   const double* vy, const double* rho) {
  auto* q = static_cast<SimD*>(s);
  q->t = t;
  for (int i = 0; i < q->Nf; ++i) {
    q->x[i] = x[i]; q->y[i] = y[i]; q->vx[i] = vx[i]; q->vy[i] = vy[i]; q->rho[i] = rho[i];
    q->e[i] = 0.0;
  }
  q->dt_prev = 0.0;
  for (int k = 0; k < q->N(); ++k) q->order[k] = k;
}
int orc_probe_rows(void* s) {
  auto* q = static_cast<SimD*>(s);
  return (int)(q->probe_rows.size() / (2 + q->P.n_probes));
}
void orc_get_probes(void* s, double* t, double* dt, double* p) {
  auto* q = static_cast<SimD*>(s);
  const int w = 2 + q->P.n_probes, rows = orc_probe_rows(s);
  for (int r = 0; r < rows; ++r) {
    t[r] = q->probe_rows[r * w];
    dt[r] = q->probe_rows[r * w + 1];
    for (int k = 0; k < q->P.n_probes; ++k) p[r * q->P.n_probes + k] = q->probe_rows[r * w + 2 + k];
  }
}
int orc_diag_rows(void* s) { return (int)(static_cast<SimD*>(s)->diag_rows.size() / ORC_NDIAG); }
void orc_get_diags(void* s, double* rows) {
  auto* q = static_cast<SimD*>(s);
  std::copy(q->diag_rows.begin(), q->diag_rows.end(), rows);
}
double orc_impulse(void* s) { return static_cast<SimD*>(s)->J; }

void orc_eval_rates(void* s, double* drho, double* ax, double* ay, double* Vx, double* Vy,
                    double* gp, double* grho, double* gvx, double* gvy, double* vmax) {
  auto* q = static_cast<SimD*>(s);
  std::vector<double> pf, D(q->Nf), a(q->Nf), b(q->Nf), c(q->Nf), d(q->Nf);
  q->prepare(q->t, pf);
  q->rates(pf, D, a, b, c, d);
  for (int i = 0; i < q->Nf; ++i) { drho[i] = D[i]; ax[i] = a[i]; ay[i] = b[i]; Vx[i] = c[i]; Vy[i] = d[i]; }
  const int NG = q->Nw + q->Nd;
  for (int g = 0; g < NG; ++g) {
    if (gp) gp[g] = q->gp[g];
    if (grho) grho[g] = q->grho[g];
    if (gvx) gvx[g] = q->gvx[g];
    if (gvy) gvy[g] = q->gvy[g];
  }
  if (vmax) *vmax = q->vmax_now();
}
void orc_eval_density(void* s, double* rho, double* p) {
  auto* q = static_cast<SimD*>(s);
  if (q->P.scheme == 1) {
    q->place_disk(q->t);
    q->build_cells();
    q->sum_density();
  }
  std::vector<double> pf;
  q->fluid_pressure(pf);
  for (int i = 0; i < q->Nf; ++i) {
    rho[i] = q->rho[i];
    p[i] = pf[i];
  }
}
void orc_get_energy(void* s, double* e) {
  auto* q = static_cast<SimD*>(s);
  for (int i = 0; i < q->Nf; ++i) e[i] = q->e[i];
}
double orc_eos_pe(const orc_params* p, double rho, double e) {
  Coef<double> k;
  k.c0 = p->c0; k.B = p->rho0 * p->c0 * p->c0 / p->gamma; k.alpha = p->alpha; k.delta = p->delta;
  return eos_p(rho, *p, k, e);
}
double orc_lattice_mass(const orc_params* p) {
  orc_params q = *p;
  q.scheme = 1;
  return make_geom(q).m_fluid;
}
void orc_audit_rates(void* s, double* out) {
  auto* q = static_cast<SimD*>(s);
  for (int k = 0; k < 4; ++k) out[k] = q->audit_rate[k];
}
void orc_get_ghosts(void* s, double* gx, double* gy, double* gm) {
  auto* q = static_cast<SimD*>(s);
  for (int g = 0; g < q->Nw + q->Nd; ++g) { gx[g] = q->gx[g]; gy[g] = q->gy[g]; gm[g] = q->gm[g]; }
}
void orc_get_order(void* s, int* order, int* cell_start) {
  auto* q = static_cast<SimD*>(s);
  std::copy(q->order.begin(), q->order.end(), order);
  std::copy(q->cell_start.begin(), q->cell_start.end(), cell_start);
}
void orc_kinematics(void* s, double t, double* x, double* v, double* a) {
  auto* q = static_cast<SimD*>(s);
  q->kin(t, x, v, a);
}
void orc_set_kin_table(void* s, int n, const double* rows) {
  auto* q = static_cast<SimD*>(s);
  q->kin_tab.assign(rows, rows + 4 * (n > 0 ? n : 0));
}
void orc_disk_state(void* s, double* x, double* v, double* a) { static_cast<SimD*>(s)->current_disk(x, v, a); }

// ---- building blocks --------------------------------------------------------
void orc_kernel(double q, double h, double* W, double* F) { orc_kernel_type(0, q, h, W, F); }
void orc_kernel_type(int type, double q, double h, double* W, double* F) {
  orc_params p;
  std::memset(&p, 0, sizeof p);
  p.dx = h; p.h_over_dx = 1.0; p.rho0 = 1.0; p.L = p.W = 1.0; p.kernel_type = type;
  Geom g = make_geom(p);
  if (!(q < 2.0)) { *W = 0; *F = 0; return; }
  kernel_WF(q, g, *W, *F);
}

void orc_eos(const orc_params* p, double rho, double* pres, double* c) {
  Coef<double> k;
  k.c0 = p->c0; k.B = p->rho0 * p->c0 * p->c0 / p->gamma; k.alpha = p->alpha; k.delta = p->delta;
  *pres = eos_p(rho, *p, k);
  *c = eos_c(rho, *p, k);
}

double orc_eos_rho(const orc_params* p, double pres) {
  Coef<double> k;
  k.c0 = p->c0; k.B = p->rho0 * p->c0 * p->c0 / p->gamma; k.alpha = p->alpha; k.delta = p->delta;
  return eos_rho(pres, *p, k);
}

double orc_elastic_energy(const orc_params* p, double rho) {
  SimD s;
  s.P = *p;
  s.set_coef(p->alpha, p->delta, p->c0);
  return s.e_el(rho);
}

double orc_cfl_dt(double cfl, double h, double c0, double vmax) { return cfl * h / (c0 + vmax); }

int orc_cell_list(const orc_params* p, int n, const double* x, const double* y, int* keys,
                  int* perm, int* cell_start) {
  Geom g = make_geom(*p);
  const int nc = g.ncx * g.ncy;
  std::vector<int> k(n), ord(n);
  for (int i = 0; i < n; ++i) {
    k[i] = cell_coord(y[i], g.y_lo, g.dc, g.ncy) * g.ncx + cell_coord(x[i], g.x_lo, g.dc, g.ncx);
    ord[i] = i;
    if (keys) keys[i] = k[i];
  }
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return k[a] < k[b]; });
  if (perm) std::copy(ord.begin(), ord.end(), perm);
  if (cell_start) {
    std::fill(cell_start, cell_start + nc + 1, 0);
    for (int i = 0; i < n; ++i) cell_start[k[i] + 1]++;
    for (int c = 1; c <= nc; ++c) cell_start[c] += cell_start[c - 1];
  }
  return nc;
}

long orc_brute_pairs(const orc_params* p, int n, const double* x, const double* y, int* out, long cap) {
  const double h = p->h_over_dx * p->dx, s2 = 4.0 * h * h;
  long m = 0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double rx = x[i] - x[j], ry = y[i] - y[j];
      if (rx * rx + ry * ry < s2) {
        if (out && m < cap) { out[2 * m] = i; out[2 * m + 1] = j; }
        ++m;
      }
    }
  return m;
}

long orc_cell_pairs(const orc_params* p, int n, const double* x, const double* y, int* out, long cap) {
  Geom g = make_geom(*p);
  const double s2 = 4.0 * g.h * g.h;
  std::vector<int> keys(n), perm(n), cs(g.ncx * g.ncy + 1);
  orc_cell_list(p, n, x, y, keys.data(), perm.data(), cs.data());
  long m = 0;
  for (int i = 0; i < n; ++i) {
    int cx = keys[i] % g.ncx, cy = keys[i] / g.ncx;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dxx = -1; dxx <= 1; ++dxx) {
        int xx = cx + dxx, yy = cy + dy;
        if (xx < 0 || xx >= g.ncx || yy < 0 || yy >= g.ncy) continue;
        int K = yy * g.ncx + xx;
        for (int k = cs[K]; k < cs[K + 1]; ++k) {
          int j = perm[k];
          if (j <= i) continue;
          double rx = x[i] - x[j], ry = y[i] - y[j];
          if (rx * rx + ry * ry < s2) {
            if (out && m < cap) { out[2 * m] = i; out[2 * m + 1] = j; }
            ++m;
          }
        }
      }
  }
  return m;
}

void orc_neighbour_stats(const orc_params* p, int n, const double* x, const double* y,
                         const int* ids, double tol, int* count, long long* idsum, int* border) {
  Geom g = make_geom(*p);
  const double s2 = 4.0 * g.h * g.h;
  std::vector<int> keys(n), perm(n), cs(g.ncx * g.ncy + 1);
  orc_cell_list(p, n, x, y, keys.data(), perm.data(), cs.data());
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    int cx = keys[i] % g.ncx, cy = keys[i] / g.ncx;
    int c = 0, b = 0;
    long long sm = 0;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dxx = -1; dxx <= 1; ++dxx) {
        int xx = cx + dxx, yy = cy + dy;
        if (xx < 0 || xx >= g.ncx || yy < 0 || yy >= g.ncy) continue;
        int K = yy * g.ncx + xx;
        for (int k = cs[K]; k < cs[K + 1]; ++k) {
          int j = perm[k];
          if (j == i) continue;
          double rx = x[i] - x[j], ry = y[i] - y[j], r2 = rx * rx + ry * ry;
          if (std::fabs(r2 - s2) < tol * s2) ++b;
          if (r2 < s2) { ++c; sm += ids[j]; }
        }
      }
    count[i] = c; idsum[i] = sm; border[i] = b;
  }
}

void orc_ghost_point(const orc_params* p, double gx, double gy, const double* vw, const double* aw,
                     int nf, const double* x, const double* y, const double* vx, const double* vy,
                     const double* rho, const double* pres, double* pg, double* rhog, double* vg) {
  Geom g = make_geom(*p);
  double SW = 0, Sp = 0, Srx = 0, Sry = 0, Svx = 0, Svy = 0;
  for (int j = 0; j < nf; ++j) {
    double rx = gx - x[j], ry = gy - y[j], r2 = rx * rx + ry * ry;
    if (!(r2 < 4.0 * g.h * g.h)) continue;
    double W, F;
    kernel_WF(std::sqrt(r2) / g.h, g, W, F);
    SW += W; Sp += pres[j] * W; Srx += rho[j] * rx * W; Sry += rho[j] * ry * W;
    Svx += vx[j] * W; Svy += vy[j] * W;
  }
  double q, ux, uy;
  if (SW > 0) {
    q = (Sp + (0.0 - aw[0]) * Srx + (p->gravity_y - aw[1]) * Sry) / SW;
    ux = 2.0 * vw[0] - Svx / SW;
    uy = 2.0 * vw[1] - Svy / SW;
  } else {
    q = 0; ux = vw[0]; uy = vw[1];
  }
  if (q < p->p_cav) q = p->p_cav;
  Coef<double> k;
  k.c0 = p->c0; k.B = p->rho0 * p->c0 * p->c0 / p->gamma;
  *pg = q;
  *rhog = p->ghost_rho_mode == 0 ? p->rho0 * (1.0 + q / (p->rho0 * p->c0 * p->c0)) : eos_rho(q, *p, k);
  vg[0] = ux; vg[1] = uy;
}

void orc_pair_rates(const orc_params* p, int n, const double* x, const double* y, const double* vx,
                    const double* vy, const double* rho, const double* pres, const double* m,
                    const int* kind, double* drho, double* ax, double* ay, double* Vx, double* Vy) {
  Geom g = make_geom(*p);
  Coef<double> k;
  k.alpha = p->alpha; k.delta = p->delta; k.c0 = p->c0; k.B = p->rho0 * p->c0 * p->c0 / p->gamma;
  auto view = [&](int j) {
    PV<double> v;
    v.x = x[j]; v.y = y[j]; v.vx = vx[j]; v.vy = vy[j]; v.rho = rho[j];
    v.P = pres[j] / (rho[j] * rho[j]);
    v.c = eos_c(rho[j], *p, k);
    v.m = m[j]; v.kind = kind[j];
    return v;
  };
  for (int i = 0; i < n; ++i) {
    if (kind[i] != 0) continue;
    PV<double> a = view(i);
    Acc<double> acc;
    for (int j = 0; j < n; ++j)
      if (j != i) pair_law(a, view(j), *p, g, k, acc);
    drho[i] = acc.D; ax[i] = acc.ax; ay[i] = acc.ay + p->gravity_y;
    Vx[i] = vx[i] + acc.Vx; Vy[i] = vy[i] + acc.Vy;
  }
}

}  // extern "C"

// The value of a state component rounded to float32 (the tangent is kept).
template <class T>
void round_value_f32(T& x) {
  x.v = (double)(float)x.v;
}
// A position rounded to the FP32 representation of the hot path: the index
// of its cell of edge dc from lo, plus a float32 offset inside the cell.
template <class T>
void round_position_f32(T& x, double lo, double dc) {
  const double c = std::floor((x.v - lo) / dc);
  double o = (double)(float)(x.v - lo - c * dc);
  double cc = c;
  if (o >= (double)(float)dc) { cc += 1.0; o = 0.0; }
  x.v = lo + cc * dc + o;
}

void tangent_run(const orc_params* p, int n_steps, const double* dt, bool round_f32, double* J, double* dJ) {
  // coupled: not differentiated; table: not held here; scheme 1 and the axisymmetric form: not built
  if (p->kin_mode == 2 || p->kin_mode == 3 || p->scheme == 1 || p->axisym) {
    *J = dJ[0] = dJ[1] = dJ[2] = std::nan("");
    return;
  }
  using D3 = Dual<3>;
  Sim<D3> s;
  s.P = *p;
  D3 a(p->alpha), d(p->delta), c(p->c0);
  a.d[0] = 1.0; d.d[1] = 1.0; c.d[2] = 1.0;
  s.set_coef(a, d, c);
  s.setup(*p, 0, nullptr);
  s.dt_table.assign(dt, dt + n_steps);
  auto round_state = [&]() {
    for (int i = 0; i < s.Nf; ++i) {
      round_position_f32(s.x[i], s.G.x_lo, s.G.dc);
      round_position_f32(s.y[i], s.G.y_lo, s.G.dc);
      round_value_f32(s.vx[i]);
      round_value_f32(s.vy[i]);
      round_value_f32(s.rho[i]);
    }
  };
  if (round_f32) round_state();
  for (int k = 0; k < n_steps; ++k) {
    s.one_step();
    if (round_f32) round_state();
  }
  *J = s.J.v;
  for (int k = 0; k < 3; ++k) dJ[k] = s.J.d[k];
}

extern "C" {

void orc_tangent_J(const orc_params* p, int n_steps, const double* dt, double* J, double* dJ) {
  tangent_run(p, n_steps, dt, false, J, dJ);
}

void orc_tangent_J_f32(const orc_params* p, int n_steps, const double* dt, double* J, double* dJ) {
  tangent_run(p, n_steps, dt, true, J, dJ);
}

}  // extern "C"
