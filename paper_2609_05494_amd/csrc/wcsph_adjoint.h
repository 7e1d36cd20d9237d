// wcsph_adjoint.h -- derivatives of the pair law, the Shepard ghost state,
// the probes and the Tait EOS, used by the reverse sweep of the step
// (internal to libwcsph.so). Scalar type T is float in the kernels.
//
// Notation: particle a receives the pair law from neighbour b at
// r = r_a - r_b, v = v_a - v_b; the pair law (continuity + delta diffusion,
// pressure + Monaghan AV, Lo-Shao laminar term, XSPH) is
//   D  += m_b F (v.r) + k_d (rho_a - rho_b)/rho_b F,  k_d = 2 delta h c0 m_b [b fluid]
//   a  += lam v - m_b F (P_a + P_b + Pi) r,  lam = 4 nu0 m_b F r^2 / (den R2)
//   V  += -eps (2 m_b / R2) W v [b fluid]
//   Pi  = -alpha h (c_a + c_b) min(v.r, 0) / (den R2)
// with den = r^2 + eta^2 h^2, R2 = rho_a + rho_b, Wendland C2 W(q) and
// grad W = F r. Given the adjoints (lD, la, lV) of particle a's rates,
// pair_vjp returns the partial derivatives of
//   L = lD D + la . a + lV . V
// with respect to every input of the pair.
#pragma once

#ifndef WC_HD
#define WC_HD __host__ __device__
#endif

template <class T>
struct PairK {
  T h, inv_h, four_h2, sigma, fgrad, eta2h2, alpha, delta, two_h_c0, eps, four_nu0;
};

template <class T>
struct PairIn {
  T rx, ry, vx, vy;  // r_a - r_b, v_a - v_b
  T ra, rb, Pa, Pb, ca, cb, mb, fl;  // fl = 1 for a fluid neighbour, 0 for a ghost
};

template <class T>
struct PairGrad {
  T rx, ry;    // dL/dr (r = r_a - r_b)
  T vx, vy;    // dL/dv (v = v_a - v_b)
  T ra, rb;    // direct density dependence
  T P, c;      // dL/dP_a = dL/dP_b, dL/dc_a = dL/dc_b
  T alpha, delta, c0x;  // explicit coefficient dependence (c0 in the delta term)
};

template <class T>
WC_HD inline T wc_min0(T x) { return x < T(0) ? x : T(0); }

// Forward pair law (the same arithmetic as the step kernels), for checks.
template <class T>
WC_HD inline void pair_forward(const PairIn<T>& in, const PairK<T>& k, T& D, T& ax, T& ay, T& Vx, T& Vy,
                               T (*sqrt_fn)(T)) {
  const T r2 = in.rx * in.rx + in.ry * in.ry;
  const T q = sqrt_fn(r2) * k.inv_h;
  const T s = T(1) - T(0.5) * q, s2 = s * s;
  const T W = k.sigma * s2 * s2 * (T(2) * q + T(1));
  const T F = -k.fgrad * s2 * s;
  const T vr = in.vx * in.rx + in.vy * in.ry;
  const T R2 = in.ra + in.rb, den = r2 + k.eta2h2, inv = T(1) / (den * R2);
  const T Pi = -k.alpha * k.h * (in.ca + in.cb) * wc_min0(vr) * inv;
  const T mF = in.mb * F;
  const T kd = in.fl * k.delta * k.two_h_c0 * in.mb;
  D = mF * vr + kd * (in.ra - in.rb) / in.rb * F;
  const T sp = in.Pa + in.Pb + Pi;
  const T lam = k.four_nu0 * mF * r2 * inv;
  ax = lam * in.vx - mF * sp * in.rx;
  ay = lam * in.vy - mF * sp * in.ry;
  const T w = in.fl * k.eps * in.mb * T(2) / R2 * W;
  Vx = -w * in.vx;
  Vy = -w * in.vy;
}

// (rcp_fn: the reciprocal the caller's precision calls for; the device
// passes the hardware reciprocal, as the step kernels use)
template <class T>
WC_HD inline void pair_vjp(const PairIn<T>& in, const PairK<T>& k, T lD, T lax, T lay, T lVx, T lVy,
                           PairGrad<T>& g, T (*sqrt_fn)(T), T (*rcp_fn)(T)) {
  const T rx = in.rx, ry = in.ry, vx = in.vx, vy = in.vy;
  const T r2 = rx * rx + ry * ry;
  const T rr = sqrt_fn(r2);
  const T q = rr * k.inv_h;
  const T s = T(1) - T(0.5) * q, s2 = s * s;
  const T W = k.sigma * s2 * s2 * (T(2) * q + T(1));
  const T F = -k.fgrad * s2 * s;
  const T dF = T(1.5) * k.fgrad * s2 * k.inv_h;  // dF / d|r|
  const T vr = vx * rx + vy * ry;
  const T R2 = in.ra + in.rb, den = r2 + k.eta2h2, inv = rcp_fn(den * R2);
  const T iR2 = rcp_fn(R2), iden = inv * R2, irb = rcp_fn(in.rb);
  const T C2 = in.ca + in.cb;
  const T mv = wc_min0(vr);
  const T Pi = -k.alpha * k.h * C2 * mv * inv;
  const T Pv = vr < T(0) ? -k.alpha * k.h * C2 * inv : T(0);  // dPi / dvr
  const T mF = in.mb * F;
  const T kd = in.fl * k.delta * k.two_h_c0 * in.mb;
  const T drho = (in.ra - in.rb) * irb;
  const T sp = in.Pa + in.Pb + Pi;
  const T lam = k.four_nu0 * mF * r2 * inv;
  const T Lv = lax * vx + lay * vy;
  const T Lr = lax * rx + lay * ry;
  const T LV = lVx * vx + lVy * vy;
  const T GLV = -in.fl * k.eps * in.mb * T(2) * iR2 * W;  // dL / d(lV . v)
  const T GW = -in.fl * k.eps * in.mb * T(2) * iR2 * LV;  // dL / dW
  const T GF = lD * in.mb * vr + lD * kd * drho + Lv * k.four_nu0 * in.mb * r2 * inv - in.mb * sp * Lr;
  const T dvr = lD * mF - mF * Lr * Pv;
  const T dden = (-Lv * lam + mF * Lr * Pi) * iden;
  const T dr2 = Lv * k.four_nu0 * mF * inv + dden;
  const T dLr = -mF * sp;
  const T fr = rr > T(0) ? GF * dF * rcp_fn(rr) : T(0);
  g.rx = fr * rx + GW * F * rx + dvr * vx + T(2) * dr2 * rx + dLr * lax;
  g.ry = fr * ry + GW * F * ry + dvr * vy + T(2) * dr2 * ry + dLr * lay;
  g.vx = dvr * rx + lam * lax + GLV * lVx;
  g.vy = dvr * ry + lam * lay + GLV * lVy;
  const T T5 = GLV * LV;
  const T dR2 = (-Lv * lam + mF * Lr * Pi - T5) * iR2;
  g.ra = dR2 + lD * kd * F * irb;
  g.rb = dR2 - lD * kd * F * in.ra * irb * irb;
  g.P = -mF * Lr;
  g.c = -mF * Lr * (-k.alpha * k.h * mv * inv);
  g.alpha = -mF * Lr * (-k.h * C2 * mv * inv);
  g.delta = lD * in.fl * k.two_h_c0 * in.mb * drho * F;
  g.c0x = lD * in.fl * k.delta * T(2) * k.h * in.mb * drho * F;  // d k_d / d c0 = 2 delta h m_b
}

// Tait EOS and its derivatives for a fluid particle: p (with the cutoff),
// P = p / rho^2, c = c0 (rho/rho0)^k, and d/drho, d/dc0 of P and c
// (derivatives of the cut branch are zero).
template <class T>
struct EosD {
  T p, P, c, dp, dPdr, dcdr, dpdc0, dPdc0, dcdc0;
};

template <class T>
WC_HD inline EosD<T> eos_d(T rho, T rho0, T c0, T gamma, T p_cav, T (*pow_fn)(T, T)) {
  EosD<T> e;
  const T x = rho / rho0;
  const T B = rho0 * c0 * c0 / gamma;
  const T xg1 = pow_fn(x, gamma - T(1));
  const T praw = B * (xg1 * x - T(1));
  const bool cut = praw < p_cav;
  e.p = cut ? p_cav : praw;
  e.dp = cut ? T(0) : c0 * c0 * xg1;
  e.dpdc0 = cut ? T(0) : T(2) * praw / c0;
  e.P = e.p / (rho * rho);
  e.dPdr = e.dp / (rho * rho) - T(2) * e.p / (rho * rho * rho);
  e.dPdc0 = e.dpdc0 / (rho * rho);
  const T kc = T(0.5) * (gamma - T(1));
  e.c = c0 * pow_fn(x, kc);
  e.dcdr = kc * e.c / rho;
  e.dcdc0 = e.c / c0;
  return e;
}
