// Reverse-mode derivative (vector-Jacobian product) of one self-interaction
// application U(theta) at one site, in FP64.
//
// Forward (qlg_math.hpp): for x in {a, b},
//   y1_x = P x = x + c(n) (v^H x) v,        c(n) = (e^{-i kappa n} - 1)/n, kappa = theta g2/5,
//   y_x  = e^{-i theta g0 n} R(F) y1_x,      R = exp(-i tau F.f), tau = theta g1,
// (times e^{-i ext} with ext = theta (V + mu) when the equation carries a potential),
// with psi = a + b, n = |psi|^2, F_nu = psi^H f_nu psi, v = S psi* (all frozen
// at the input).  Cotangents follow lambda = dL/dRe z + i dL/dIm z, so for a
// complex-linear map y = M z the pull-back is lambda_z = M^H lambda_y.
//
// In the frame Q = Phi d(beta) of F (Q^H (F.f) Q = |F| f_z) everything
// diagonalises: with Y = Q^H y1, Lam = Q^H lambda_y and E_m = e^{-i(th g0 n + m phi)},
//   lambda_{y1} = Q conj(E) Lam,
//   dL/dn  (density) = th g0 sum_m Im(conj(Lam_m) E_m Y_m),
//   dL/dg0            = th n  sum_m Im(conj(Lam_m) E_m Y_m),
//   dL/dg1            = th |F| sum_m m Im(conj(Lam_m) E_m Y_m),
// and the derivative of R with respect to F is the Frechet derivative of the
// exponential, whose divided differences between neighbouring m are
// e^{-i phi (m_j + m_k)/2} sinc(phi/2) (only neighbours couple through f_x, f_y):
//   dL/dF = R3 G,  G_mu = Re(-i tau sum_jk conj(M'_jk) Delta_jk (f_mu)_jk),
//   M' = sum_x (Q^H lambda_{y2,x}) (Q^H y1_x)^H,  lambda_{y2} = e^{i th g0 n} lambda_y,
// with R3 = R_z(alpha) R_y(beta) the rotation taking z to F.  The singlet
// factor contributes, per x with s_x = v^H x and l = lambda_{y1,x},
//   lambda_x  = P^H l = l + conj(c) (v^H l) v,
//   lambda_psi += conj(c) conj(l^H v) S x* + c s_x S conj(l),
//   dL/dn += Re(c'(n) s_x (l^H v)),   dL/dg2 += Re(dc/dg2 s_x (l^H v)).
// Finally lambda_psi += 2 dL/dn psi + 2 sum_nu dL/dF_nu f_nu psi and
// lambda_a = P^H l_a + lambda_psi, lambda_b = P^H l_b + lambda_psi.
#pragma once

#include "qlg_math.hpp"

namespace qlg {

// Forward frame and phases of one application (FP64), shared by the VJP.
struct UFrame {
  cx<double> p[5];     // psi
  double n, Fx, Fy, Fz, Fn, Fperp;
  double phi0, phi;    // theta g0 n, theta g1 |F|
  cx<double> cs;       // c(n)
  cx<double> E[5];     // e^{-i (phi0 + m phi)}, m = 2..-2
  cx<double> u;        // e^{i alpha}
  cx<double> e0, eh;   // e^{-i phi0}, e^{-i phi/2}
  double sinc_hp;      // sin(phi/2) / (phi/2)
  cx<double> ekn;      // e^{-i kappa n}, kappa = theta g2 / 5
  double ca, sa, cb, sb;
  DBlocks<double> d;   // d^2(beta) in the blocks of d_apply (qlg_math.hpp)
};

// ext: theta (V + mu) of a psi-independent term (V(x) + mu) psi_m in the equation of
// motion; it joins the density phase phi0 and, not depending on psi, adds nothing
// to the derivatives with respect to n, F or the couplings.
// kUniform: when the three angles (phi0, phi/2 and the singlet's kappa n / 2) are at most
// 1/16 on every lane of the wavefront, all lanes take the short sine/cosine series without a
// per-lane branch (one uniform test), sin(x)/x from the same polynomials, and the frame as
// selects: for kernels that run one wavefront per SIMD, where every branch instruction costs
// an issue slot of the VALU.  The results are those of the per-lane form to rounding.
template <bool kUniform = false>
QLG_HD void u_frame(const cx<double> (&a)[5], const cx<double> (&b)[5], double theta, double g0,
                    double g1, double g2, UFrame& f, double ext = 0.0) {
  const double r6 = Consts::r6;
  double q[5];
  for (int m = 0; m < 5; ++m) {
    f.p[m] = a[m] + b[m];
    q[m] = f.p[m].re * f.p[m].re + f.p[m].im * f.p[m].im;
  }
  f.n = q[0] + q[1] + q[2] + q[3] + q[4];
  f.Fz = 2.0 * (q[0] - q[4]) + (q[1] - q[3]);
  const cx<double> f1 = cmulc(f.p[0], f.p[1]) + cmulc(f.p[3], f.p[4]);
  const cx<double> f2 = cmulc(f.p[1], f.p[2]) + cmulc(f.p[2], f.p[3]);
  f.Fx = 2.0 * f1.re + r6 * f2.re;
  f.Fy = 2.0 * f1.im + r6 * f2.im;
  const double Fp2 = f.Fx * f.Fx + f.Fy * f.Fy;
  const double Fn2 = Fp2 + f.Fz * f.Fz;
  // |F|, F_perp and their reciprocals (below the normal range the frame is immaterial: phi ~ 0)
  const double tiny2 = 1e-300;
  const bool has_F = Fn2 > tiny2, has_perp = Fp2 > tiny2;
  double iP, iF;
  if constexpr (kUniform) {
    const double rP = rsqrt_t(has_perp ? Fp2 : 1.0), rF = rsqrt_t(has_F ? Fn2 : 1.0);
    iP = has_perp ? rP : 0.0;
    iF = has_F ? rF : 0.0;
  } else {
    iP = has_perp ? rsqrt_t(Fp2) : 0.0;
    iF = has_F ? rsqrt_t(Fn2) : 0.0;
  }
  f.Fperp = Fp2 * iP;
  f.Fn = Fn2 * iF;
  f.phi0 = theta * g0 * f.n + ext;
  f.phi = theta * g1 * f.Fn;
  // c(n) = (e^{-i kappa n} - 1)/n = kappa sinc(h) (-sin h - i cos h), h = kappa n / 2
  const double kappa = theta * g2 * 0.2, h = 0.5 * kappa * f.n;
  const double hp = 0.5 * f.phi;
  double s0, c0, s1, c1, sh, ch, sinc;
  if (kUniform && all_lanes(fmax(fmax(fabs(f.phi0), fabs(hp)), fabs(h)) <= 0.0625)) {
    double x0;
    sincos_short(f.phi0, &s0, &c0, &x0);
    sincos_short(hp, &s1, &c1, &f.sinc_hp);
    sincos_short(h, &sh, &ch, &sinc);
  } else {
    sincos_t(f.phi0, &s0, &c0);
    sincos_t(hp, &s1, &c1);
    sincos_t(h, &sh, &ch);
    sinc = fabs(h) < 1e-4 ? 1.0 - h * h * (1.0 / 6.0) : sh * rcp_t(h);
    f.sinc_hp = fabs(hp) < 1e-4 ? 1.0 - hp * hp * (1.0 / 6.0) : s1 * rcp_t(hp);
  }
  // E_m = e^{-i phi0} (e^{-i phi})^m from two phases: e^{-i phi0} and eh = e^{-i phi/2}
  {
    const cx<double> e0{c0, -s0}, eh{c1, -s1}, e1 = eh * eh;
    f.E[2] = e0;
    f.E[1] = e0 * e1;
    f.E[0] = f.E[1] * e1;
    f.E[3] = e0 * conj(e1);
    f.E[4] = f.E[3] * conj(e1);
    f.e0 = e0;
    f.eh = eh;
  }
  f.cs = cx<double>{-kappa * sinc * sh, -kappa * sinc * ch};
  f.ekn = cx<double>{ch, -sh} * cx<double>{ch, -sh};   // e^{-i kappa n}
  // frame (F_perp = 0: beta = 0 or pi exactly, as in the forward)
  if constexpr (kUniform) {
    f.ca = has_perp ? f.Fx * iP : 1.0;
    f.sa = has_perp ? f.Fy * iP : 0.0;
    const double cz = f.Fz >= 0 ? 1.0 : -1.0, cp = f.Fz * iF;
    const double cf = has_perp ? cp : cz;
    f.cb = has_F ? cf : 1.0;
    f.sb = f.Fperp * iF;   // 0 without F
  } else {
    f.ca = 1.0; f.sa = 0.0; f.cb = 1.0; f.sb = 0.0;
    if (has_perp) { f.ca = f.Fx * iP; f.sa = f.Fy * iP; }
    if (has_F) {
      f.cb = has_perp ? f.Fz * iF : (f.Fz >= 0 ? 1.0 : -1.0);
      f.sb = f.Fperp * iF;
    }
  }
  f.u = cx<double>{f.ca, f.sa};
  f.d = d_blocks(f.cb, f.sb);
}

// Q^H x = d^T Phi^* x (Phi^* multiplies component m by u^m)
QLG_HD void to_frame(const UFrame& f, const cx<double> (&x)[5], cx<double> (&out)[5]) {
  const cx<double> u = f.u, u2 = u * u, uc = conj(u), u2c = conj(u2);
  const cx<double> w[5] = {x[0] * u2, x[1] * u, x[2], x[3] * uc, x[4] * u2c};
  d_apply<double, true>(f.d, w, out);
}

// Q z = Phi d z
QLG_HD void from_frame(const UFrame& f, const cx<double> (&z)[5], cx<double> (&out)[5]) {
  const cx<double> u = f.u, u2 = u * u, uc = conj(u), u2c = conj(u2);
  cx<double> t[5];
  d_apply<double, false>(f.d, z, t);
  out[0] = t[0] * u2c;
  out[1] = t[1] * uc;
  out[2] = t[2];
  out[3] = t[3] * u;
  out[4] = t[4] * u2;
}

// (S z)_m = (-1)^m z_{-m}
QLG_HD void apply_S(const cx<double> (&z)[5], cx<double> (&out)[5]) {
  out[0] = z[4];
  out[1] = -1.0 * z[3];
  out[2] = z[2];
  out[3] = -1.0 * z[1];
  out[4] = z[0];
}

// c'(n) for c(n) = (e^{-i k n} - 1)/n; e = e^{-i k n}.  For |k n| < 0.1 the series
// c'(n) = sum_{j>=2} (-i k)^j (j-1) n^{j-2} / j! = (-i k)^2 sum_{q>=0} (q+1)/(q+2)! (-i z)^q,
// z = k n, truncated after q = 12 (the next term is below 1e-24): its real and imaginary
// parts are the even and odd powers of z, two polynomials in z^2.
template <bool kUniform = false>
QLG_HD cx<double> dc_dn(double kappa, double n, cx<double> e) {
  const double z = kappa * n;
  auto series = [&]() {
    const double y = z * z;
    // (q+1)/(q+2)! for q = 0..12, alternating in sign within each parity
    const double pe = 1.0 / 2 + y * (-1.0 / 8 + y * (1.0 / 144 + y * (-1.0 / 5760 + y * (1.0 / 403200 +
                      y * (-1.0 / 43545600 + y * (1.0 / 6706022400.0))))));
    const double po = 1.0 / 3 + y * (-1.0 / 30 + y * (1.0 / 840 + y * (-1.0 / 45360 + y * (1.0 / 3991680 +
                      y * (-1.0 / 518918400.0)))));
    const double k2 = kappa * kappa;
    return cx<double>{-k2 * pe, k2 * z * po};   // -k^2 (pe - i z po)
  };
  const bool small = fabs(z) < 0.1;
  if constexpr (kUniform) {
    if (all_lanes(small)) return series();   // the usual case, without a per-lane branch
  }
  if (small) return series();
  const double in = rcp_t(n);
  const cx<double> cn = in * (e - cx<double>{1.0, 0.0});
  const cx<double> t = cx<double>{0.0, -kappa} * e;            // -i k e^{-ikn}
  return in * (t - cn);
}

// In: a, b (input of U), la, lb (cotangents of U's outputs).
// Out: la, lb replaced by cotangents of a, b; dg[0..2] incremented.
template <bool kUniform = false>
QLG_HD void potential_vjp(const cx<double> (&a)[5], const cx<double> (&b)[5], cx<double> (&la)[5],
                          cx<double> (&lb)[5], double theta, double g0, double g1, double g2, double (&dg)[3],
                          double ext = 0.0) {
  UFrame f;
  u_frame<kUniform>(a, b, theta, g0, g1, g2, f, ext);
  const double tau = theta * g1;
  cx<double> v[5];
  {
    cx<double> pc[5];
    for (int m = 0; m < 5; ++m) pc[m] = conj(f.p[m]);
    apply_S(pc, v);                          // v = S psi*
  }
  double dn = 0.0;                           // dL/dn
  // G in the frame, G_mu = Re(-i tau sum_jk conj(M'_jk) Delta_jk (f_mu)_jk), accumulated over a
  // and b: only the diagonal (f_z) and the first off-diagonals (f_x, f_y) of M' enter
  double dFx = 0.0, dFy = 0.0, dGz = 0.0;
  cx<double> lpsi[5] = {};
  const double cfac[4] = {2.0, Consts::r6, Consts::r6, 2.0};
  const double sc = f.sinc_hp;   // sinc(phi/2)
  // divided differences between neighbouring m: Delta = e^{-i phi0} e^{-i phi (m_i + m_{i+1})/2} sinc(phi/2),
  // m_i + m_{i+1} = 3, 1, -1, -3: powers of eh = e^{-i phi/2}
  cx<double> dlt[4];
  {
    const cx<double> w1 = sc * (f.e0 * f.eh), w3 = w1 * (f.eh * f.eh);
    const cx<double> v1 = sc * (f.e0 * conj(f.eh)), v3 = v1 * conj(f.eh * f.eh);
    dlt[0] = w3;
    dlt[1] = w1;
    dlt[2] = v1;
    dlt[3] = v3;
  }
  const double kappa = theta * g2 * 0.2;
  const cx<double> dcn = dc_dn<kUniform>(kappa, f.n, f.ekn);
  const cx<double> dcg = cx<double>{0.0, -theta * 0.2} * f.ekn;
  // one 5-vector x; l holds the output cotangent on entry and P^H lambda_{y1} on exit
  auto one = [&](const cx<double>(&x)[5], cx<double>(&l)[5]) {
    cx<double> s{0.0, 0.0};
    for (int m = 0; m < 5; ++m) s = s + cmulc(v[m], x[m]);    // v^H x
    cx<double> Y[5], Lam[5];
    {
      cx<double> y1[5];
      for (int m = 0; m < 5; ++m) y1[m] = x[m] + (f.cs * s) * v[m];
      to_frame(f, y1, Y);
    }
    to_frame(f, l, Lam);
    double acc0 = 0.0, acc1 = 0.0;
    for (int i = 0; i < 5; ++i) {
      const double t = (f.E[i] * cmulc(Lam[i], Y[i])).im;     // Im(conj(Lam) E Y)
      acc0 += t;
      acc1 += (2 - i) * t;
    }
    dn += theta * g0 * acc0;
    dg[0] += theta * f.n * acc0;
    dg[1] += theta * f.Fn * acc1;
    dGz += acc1;                                               // Re(-i z) = Im(z)
    for (int i = 0; i < 4; ++i) {
      const cx<double> tu = dlt[i] * cmulc(Lam[i], Y[i + 1]);   // conj(M'_{i,i+1}) Delta
      const cx<double> td = dlt[i] * cmulc(Lam[i + 1], Y[i]);   // conj(M'_{i+1,i}) Delta
      const double ch = 0.5 * cfac[i];
      // f_x: (i,i+1) and (i+1,i) entries ch;  f_y: (i,i+1) = -i ch, (i+1,i) = +i ch
      dFx += ch * (tu.im + td.im);
      dFy += ch * (td.re - tu.re);
    }
    // cotangent of y1: Q conj(E) Lam (reusing Y for it)
    for (int i = 0; i < 5; ++i) Lam[i] = conj(f.E[i]) * Lam[i];
    from_frame(f, Lam, Y);
    // singlet factor
    cx<double> lv{0.0, 0.0};
    for (int m = 0; m < 5; ++m) lv = lv + cmulc(Y[m], v[m]);   // l^H v
    const cx<double> k1 = conj(f.cs) * conj(lv), k2 = f.cs * s;
    for (int m = 0; m < 5; ++m) {
      l[m] = Y[m] + k1 * v[m];
      // (S z)_m = (-1)^m z_{-m}: index i <-> 4 - i, sign - for m = +-1
      const double sg = (m == 1 || m == 3) ? -1.0 : 1.0;
      lpsi[m] = lpsi[m] + sg * (k1 * conj(x[4 - m]) + k2 * conj(Y[4 - m]));
    }
    dn += (dcn * s * lv).re;
    dg[2] += (dcg * s * lv).re;
  };
  one(a, la);
  one(b, lb);
  dGz *= tau;
  dFx *= tau;
  dFy *= tau;
  // lab frame: dL/dF = R3 G,  R3 = R_z(alpha) R_y(beta)
  const double ca = f.ca, sa = f.sa, cb = f.cb, sb = f.sb;
  const double LFx = ca * cb * dFx - sa * dFy + ca * sb * dGz;
  const double LFy = sa * cb * dFx + ca * dFy + sa * sb * dGz;
  const double LFz = -sb * dFx + cb * dGz;
  // lambda_psi += 2 dn psi + 2 (LFz f_z + (LFx - i LFy)/2 f_+ + (LFx + i LFy)/2 f_-) psi
  cx<double> fp[5] = {}, fm[5] = {};
  for (int i = 0; i < 4; ++i) {
    fp[i] = cfac[i] * f.p[i + 1];       // (f_+ psi)_i
    fm[i + 1] = cfac[i] * f.p[i];       // (f_- psi)_{i+1}
  }
  const cx<double> cpl{0.5 * LFx, -0.5 * LFy}, cmi{0.5 * LFx, 0.5 * LFy};
  for (int i = 0; i < 5; ++i) {
    const cx<double> fz = (double)(2 - i) * f.p[i];
    cx<double> t = (2.0 * dn) * f.p[i] + (2.0 * LFz) * fz;
    t = t + 2.0 * (cpl * fp[i] + cmi * fm[i]);
    lpsi[i] = lpsi[i] + t;
  }
  for (int m = 0; m < 5; ++m) {
    la[m] = la[m] + lpsi[m];
    lb[m] = lb[m] + lpsi[m];
  }
}

}  // namespace qlg
