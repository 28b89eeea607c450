// Per-site arithmetic of the spin-2 QLG step: collide and the self-interaction U.
//
// Everything here is __host__ __device__ so that the same code can be
// exercised on the CPU before it runs on gfx950.
//
// Component order inside a site: index 0..4 <-> m_f = 2, 1, 0, -1, -2.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#define QLG_HD __host__ __device__ __forceinline__

namespace qlg {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T> QLG_HD cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> QLG_HD cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> QLG_HD cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> QLG_HD cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> QLG_HD cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> QLG_HD cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename T> QLG_HD cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// acc + a * b
template <typename T> QLG_HD cx<T> cfma(cx<T> a, cx<T> b, cx<T> acc) {
  return {acc.re + a.re * b.re - a.im * b.im, acc.im + a.re * b.im + a.im * b.re};
}
// c ? x : y, component-wise (a select of values, never of addresses)
template <typename T> QLG_HD cx<T> sel(bool c, cx<T> x, cx<T> y) {
  return {c ? x.re : y.re, c ? x.im : y.im};
}
// acc + s * a (s real)
template <typename T> QLG_HD cx<T> rfma(T s, cx<T> a, cx<T> acc) {
  return {acc.re + s * a.re, acc.im + s * a.im};
}

// sin and cos of x.  The phase angles of U are small (|x| << 1 for any stable
// time step), so |x| <= pi/4 is evaluated by the Taylor series itself, with
// enough terms that the truncation (|x|^11/11! ~ 2e-9 in FP32, |x|^19/19! ~ 1e-19
// in FP64 at |x| = pi/4) stays below the format's rounding; larger angles take
// the library routine.  Below |x| = 1/16, where the angles of a typical step lie,
// fewer terms reach the same bound: the first omitted terms are |x|^7/7! and
// |x|^8/8! (FP32; < 1e-12 |x|) and |x|^11/11! and |x|^10/10! (FP64; < 1e-19 |x|).
QLG_HD void sincos_t(float x, float* s, float* c) {
  if (fabsf(x) <= 0.0625f) {
    const float x2 = x * x;
    *s = x * (1.0f + x2 * (-1.0f / 6 + x2 * (1.0f / 120)));
    *c = 1.0f + x2 * (-0.5f + x2 * (1.0f / 24 + x2 * (-1.0f / 720)));
  } else if (fabsf(x) <= 0.78539816f) {
    const float x2 = x * x;
    *s = x * (1.0f + x2 * (-1.0f / 6 + x2 * (1.0f / 120 + x2 * (-1.0f / 5040 + x2 * (1.0f / 362880)))));
    *c = 1.0f + x2 * (-0.5f + x2 * (1.0f / 24 + x2 * (-1.0f / 720 + x2 * (1.0f / 40320 + x2 * (-1.0f / 3628800)))));
  } else {
    sincosf(x, s, c);
  }
}
QLG_HD void sincos_t(double x, double* s, double* c) {
  if (fabs(x) <= 0.0625) {
    const double x2 = x * x;
    double ps = 1.0 / 362880.0, pc = 1.0 / 40320.0;   // 1/9!, 1/8!
    ps = fma(x2, ps, -1.0 / 5040.0);
    pc = fma(x2, pc, -1.0 / 720.0);
    ps = fma(x2, ps, 1.0 / 120.0);
    pc = fma(x2, pc, 1.0 / 24.0);
    ps = fma(x2, ps, -1.0 / 6.0);
    pc = fma(x2, pc, -0.5);
    *s = fma(x * x2, ps, x);
    *c = fma(x2, pc, 1.0);
  } else if (fabs(x) <= 0.7853981633974483) {
    const double x2 = x * x;
    double ps = 1.0 / 355687428096000.0, pc = 1.0 / 20922789888000.0;   // 1/17!, 1/16!
    ps = fma(x2, ps, -1.0 / 1307674368000.0);    // 1/15!
    pc = fma(x2, pc, -1.0 / 87178291200.0);      // 1/14!
    ps = fma(x2, ps, 1.0 / 6227020800.0);        // 1/13!
    pc = fma(x2, pc, 1.0 / 479001600.0);         // 1/12!
    ps = fma(x2, ps, -1.0 / 39916800.0);         // 1/11!
    pc = fma(x2, pc, -1.0 / 3628800.0);          // 1/10!
    ps = fma(x2, ps, 1.0 / 362880.0);            // 1/9!
    pc = fma(x2, pc, 1.0 / 40320.0);             // 1/8!
    ps = fma(x2, ps, -1.0 / 5040.0);             // 1/7!
    pc = fma(x2, pc, -1.0 / 720.0);              // 1/6!
    ps = fma(x2, ps, 1.0 / 120.0);               // 1/5!
    pc = fma(x2, pc, 1.0 / 24.0);                // 1/4!
    ps = fma(x2, ps, -1.0 / 6.0);
    pc = fma(x2, pc, -0.5);
    *s = fma(x * x2, ps, x);
    *c = fma(x2, pc, 1.0);
  } else {
    sincos(x, s, c);
  }
}
// sin x, cos x and sin(x)/x for |x| <= 1/16 by the short series of sincos_t (sin(x)/x is
// 1 + x^2 ps, the polynomial of the sine before its final multiply-add): no branch, and
// no division for sin(x)/x.
QLG_HD void sincos_short(float x, float* s, float* c, float* sx) {
  const float x2 = x * x;
  const float ps = -1.0f / 6 + x2 * (1.0f / 120);
  *sx = 1.0f + x2 * ps;
  *s = x * *sx;
  *c = 1.0f + x2 * (-0.5f + x2 * (1.0f / 24 + x2 * (-1.0f / 720)));
}
QLG_HD void sincos_short(double x, double* s, double* c, double* sx) {
  const double x2 = x * x;
  double ps = 1.0 / 362880.0, pc = 1.0 / 40320.0;
  ps = fma(x2, ps, -1.0 / 5040.0);
  pc = fma(x2, pc, -1.0 / 720.0);
  ps = fma(x2, ps, 1.0 / 120.0);
  pc = fma(x2, pc, 1.0 / 24.0);
  ps = fma(x2, ps, -1.0 / 6.0);
  pc = fma(x2, pc, -0.5);
  *sx = fma(x2, ps, 1.0);
  *s = fma(x * x2, ps, x);
  *c = fma(x2, pc, 1.0);
}

// Whether p holds on every active lane of the wavefront (the host build: p itself).  A
// branch on it is uniform: no execution-mask changes, both sides never run.
QLG_HD bool all_lanes(bool p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_ballot_w64(!p) == 0;
#else
  return p;
#endif
}

QLG_HD float sqrt_t(float x) { return sqrtf(x); }
QLG_HD double sqrt_t(double x) { return sqrt(x); }

// 1/sqrt(x) for x > 0 and 1/x for x != 0 (normal): the hardware approximations
// (about one ulp) in FP32; in FP64 the hardware estimate refined by two Newton
// steps, each of which squares its relative error (y <- y + y (1 - x y^2) / 2 and
// y <- y + y (1 - x y)), to within a few ulp of the exact value (the host build
// divides).
QLG_HD float rsqrt_t(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}
QLG_HD double rsqrt_t(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double r = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, r, y);
  }
  return y;
#else
  return 1.0 / sqrt(x);
#endif
}
QLG_HD float rcp_t(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
QLG_HD double rcp_t(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) y = fma(y, fma(-x, y, 1.0), y);
  return y;
#else
  return 1.0 / x;
#endif
}

// Angles of one application of U(theta): theta*g0, theta*g1, theta*g2/5.
template <typename T>
struct Angles {
  T tg0, tg1, tg25;
  // U may be evaluated on the state scaled by an exact power of two s (the
  // fused kernels defer the 1/4 of each I'): then tg0 and tg25 carry 1/s^2 and
  // fs = 1/s^2 brings F back to its true scale, so that W, a function of
  // theta n, theta F, the direction of F and (v v^H)/n only, is unchanged.
  T fs = T(1);
};

// ---------------------------------------------------------------------------
// Collide (sqrt SWAP on each (a_m, b_m) pair), without its factor 1/2:
//   2 a' = (a + b) - i (a - b),   2 b' = (a + b) + i (a - b).
// Two collides and one exact multiplication by 1/4 give C C exactly as the
// scaled form would (scaling by powers of two commutes with rounding); the
// fused step kernels collect the four factors 1/4 of a step's I' into one
// multiplication by 1/256 (scale_by) and evaluate U in between with Angles::fs.
// ---------------------------------------------------------------------------
template <typename T>
QLG_HD void collide2(cx<T> (&a)[5], cx<T> (&b)[5]) {
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const T sr = a[m].re + b[m].re, si = a[m].im + b[m].im;
    const T dr = a[m].re - b[m].re, di = a[m].im - b[m].im;
    a[m] = cx<T>{sr + di, si - dr};
    b[m] = cx<T>{sr - di, si + dr};
  }
}

template <typename T>
QLG_HD void scale_by(cx<T> (&a)[5], cx<T> (&b)[5], T f) {
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    a[m] = f * a[m];
    b[m] = f * b[m];
  }
}

template <typename T>
QLG_HD void scale_quarter(cx<T> (&a)[5], cx<T> (&b)[5]) {
  scale_by(a, b, T(0.25));
}

// ---------------------------------------------------------------------------
// Frozen-field self-interaction U(theta) applied to x = a and x = b:
//   x <- exp(-i th g0 n) R P x,
//   P = I + (exp(-i th g2 n/5) - 1) v v^H / n,   v_m = (-1)^m conj(psi_{-m}),
//   R = exp(-i th g1 F.f) = Phi d(beta) diag(exp(-i phi k)) d(beta)^T Phi^*,
// with psi = a + b, n = |psi|^2, F_nu = psi^H f_nu psi, phi = th g1 |F|,
// F = |F| (sin b cos al, sin b sin al, cos b), Phi = diag(exp(-i al m)) and
// d(beta) the real spin-2 rotation exp(-i beta f_y).
//
// Every factor is applied as "identity + small correction": the corrections
// use e^{-i x} - 1 = -2 sin^2(x/2) - 2i sin(x/2) cos(x/2), so the part of the
// state that the identity carries is never rounded and the norm error per
// application is second order in the phase angles.
// ---------------------------------------------------------------------------
struct Consts {
  static constexpr double r6 = 2.449489742783178098197284;    // sqrt(6)
  static constexpr double r32 = 1.224744871391589049098642;   // sqrt(3/2)
  static constexpr double r38 = 0.6123724356957945245493210;  // sqrt(3/8)
};

// Coefficients of W for one site, computed once and applied to a and to b.
//
// The real spin-2 rotation d(beta) satisfies d_{-m',-m} = (-1)^{m'-m} d_{m'm}, so it
// commutes with the flip (J x)_m = (-1)^m x_{-m} and splits into blocks on the
// combinations x_m +- x_{-m}: applied through them it takes 21 multiply-adds per
// complex 5-vector instead of 25.  In terms of c = cos beta, s = sin beta the block
// entries are
//   A = (d22 + d2-2)/2 = 1/2 - s^2/4,  B = (d22 - d2-2)/2 = (d11 + d1-1)/2 = c/2,
//   C = (d21 + d2-1)/2 = -s/2,         E = (d21 - d2-1)/2 = -s c/2,
//   G = (d11 - d1-1)/2 = c^2 - 1/2,
// with d20 = sqrt(3/8) s^2, d10 = -sqrt(3/2) s c, d00 = (3 c^2 - 1)/2.
template <typename T>
struct DBlocks {
  T dA, dB, dC, dE, dG, d20, d10, d00;
};

template <typename T>
QLG_HD DBlocks<T> d_blocks(T cb, T sb) {
  const T r32 = T(Consts::r32), r38 = T(Consts::r38);
  const T sb2 = sb * sb, cb2 = cb * cb, sbcb = sb * cb;
  DBlocks<T> D;
  D.dA = T(0.5) - T(0.25) * sb2;
  D.dB = T(0.5) * cb;
  D.dC = T(-0.5) * sb;
  D.dE = T(-0.5) * sbcb;
  D.dG = cb2 - T(0.5);
  D.d20 = r38 * sb2;
  D.d10 = -r32 * sbcb;
  D.d00 = T(1.5) * cb2 - T(0.5);
  return D;
}

template <typename T>
struct WCoef {
  cx<T> p[5];                                  // psi = a + b
  cx<T> cs;                                    // (exp(-i th g2 n/5) - 1) / n (0/0 -> -i th g2/5)
  cx<T> dl[5];                                 // exp(-i (th g0 n + k phi)) - 1, k = 2..-2
  cx<T> u, u2;                                 // e^{i alpha}, e^{2 i alpha}
  DBlocks<T> d;                                // d^2(beta) in the blocks above
};

// y = d(beta)^T x and y = d(beta) x for a complex 5-vector (m = 2..-2) through the
// blocks of WCoef: with s0 = x_2 + x_-2, t0 = x_2 - x_-2, s1 = x_1 + x_-1, t1 = x_1 - x_-1,
//   (d^T x)_{2,-2} = (A s0 - E t1 + d20 x0) +- (B t0 - C s1),
//   (d^T x)_{1,-1} = (C t0 + B s1) +- (E s0 + G t1 - d10 x0),
//   (d^T x)_0      = d20 s0 + d10 t1 + d00 x0,
//   (d x)_{2,-2}   = (A s0 + E t1 + d20 x0) +- (B t0 + C s1),
//   (d x)_{1,-1}   = (B s1 - C t0) +- (G t1 - E s0 + d10 x0),
//   (d x)_0        = d20 s0 - d10 t1 + d00 x0.
template <typename T, bool kTranspose>
QLG_HD void d_apply(const DBlocks<T>& W, const cx<T> (&x)[5], cx<T> (&y)[5]) {
  const cx<T> s0 = x[0] + x[4], t0 = x[0] - x[4], s1 = x[1] + x[3], t1 = x[1] - x[3];
  const T sgn = kTranspose ? T(-1) : T(1);
  const cx<T> P = rfma(W.d20, x[2], rfma(sgn * W.dE, t1, W.dA * s0));
  const cx<T> Q = rfma(sgn * W.dC, s1, W.dB * t0);
  const cx<T> R = rfma(-sgn * W.dC, t0, W.dB * s1);
  const cx<T> S = rfma(sgn * W.d10, x[2], rfma(W.dG, t1, (-sgn) * W.dE * s0));
  y[0] = P + Q;
  y[4] = P - Q;
  y[1] = R + S;
  y[3] = R - S;
  y[2] = rfma(W.d00, x[2], rfma(-sgn * W.d10, t1, W.d20 * s0));
}

// kExt: the equation of motion carries the psi-independent term (V(x) + mu) psi_m
// (Sec. II, "Additional terms"); ext = theta (V(x) + mu) joins the density phase.
template <typename T, bool kExt = false>
QLG_HD void w_coefficients(const cx<T> (&a)[5], const cx<T> (&b)[5], const Angles<T> ang, WCoef<T>& W,
                           T ext = T(0)) {
  const T r6 = T(Consts::r6);
  T q[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    W.p[m] = a[m] + b[m];
    q[m] = W.p[m].re * W.p[m].re + W.p[m].im * W.p[m].im;
  }
  const T n = q[0] + q[1] + q[2] + q[3] + q[4];
  const T Fz = ang.fs * (T(2) * (q[0] - q[4]) + (q[1] - q[3]));
  // F_x + i F_y = psi^H f_+ psi = 2 p2* p1 + sqrt6 p1* p0 + sqrt6 p0* p-1 + 2 p-1* p-2
  const cx<T> f1 = cmulc(W.p[0], W.p[1]) + cmulc(W.p[3], W.p[4]);
  const cx<T> f2 = cmulc(W.p[1], W.p[2]) + cmulc(W.p[2], W.p[3]);
  const T Fx = ang.fs * (T(2) * f1.re + r6 * f2.re);
  const T Fy = ang.fs * (T(2) * f1.im + r6 * f2.im);
  const T Fp2 = Fx * Fx + Fy * Fy;
  const T Fn2 = Fp2 + Fz * Fz;
  // |F|, F_perp and their reciprocals; below `tiny` the direction is immaterial
  // (phi ~ 0) and F is taken along z
  const T tiny2 = sizeof(T) == 4 ? T(1e-36) : T(1e-300);   // normal in both formats
  const bool has_F = Fn2 > tiny2, has_perp = Fp2 > tiny2;
  // (selects around unconditional evaluations: no divergent branch)
  const T rF = rsqrt_t(has_F ? Fn2 : T(1)), rp = rsqrt_t(has_perp ? Fp2 : T(1));
  const T iF = has_F ? rF : T(0);
  const T ip = has_perp ? rp : T(0);
  const T Fn = Fn2 * iF;
  const T Fperp = Fp2 * ip;

  // half-angle phases: mu = exp(-i x) - 1 = -2 sin(x/2) (sin(x/2) + i cos(x/2)).  When all
  // three half angles of every lane are at most 1/16 (the usual case) they take the short
  // series without a branch per lane, the singlet's sin(h)/h included.
  T s0, c0, s1, c1, s2, c2, sinc;
  const T h2 = T(0.5) * ang.tg25 * n;
  const T h0 = kExt ? T(0.5) * (ang.tg0 * n + ext) : T(0.5) * ang.tg0 * n;
  const T h1 = T(0.5) * ang.tg1 * Fn;
  if (all_lanes(fmax(fmax(fabs(h0), fabs(h1)), fabs(h2)) <= T(0.0625))) {
    T x0, x1;
    sincos_short(h0, &s0, &c0, &x0);
    sincos_short(h1, &s1, &c1, &x1);
    sincos_short(h2, &s2, &c2, &sinc);
  } else {
    sincos_t(h0, &s0, &c0);
    sincos_t(h1, &s1, &c1);
    sincos_t(h2, &s2, &c2);
    sinc = fabs(h2) < T(1e-4) ? T(1) - h2 * h2 * T(1.0 / 6.0) : s2 * rcp_t(h2);
  }
  const cx<T> mu0{T(-2) * s0 * s0, T(-2) * s0 * c0};
  const cx<T> mu1{T(-2) * s1 * s1, T(-2) * s1 * c1};
  // nu_k = exp(-i k phi) - 1 for k = 2, 1, -1, -2
  const cx<T> nu2 = T(2) * mu1 + mu1 * mu1;
  const cx<T> mu1c = conj(mu1), nu2c = conj(nu2);
  // E_k - 1 = exp(-i (phi0 + k phi)) - 1 = mu0 + nu_k + mu0 nu_k
  W.dl[0] = mu0 + nu2 + mu0 * nu2;
  W.dl[1] = mu0 + mu1 + mu0 * mu1;
  W.dl[2] = mu0;
  W.dl[3] = mu0 + mu1c + mu0 * mu1c;
  W.dl[4] = mu0 + nu2c + mu0 * nu2c;

  // singlet coefficient (exp(-i th g2 n/5) - 1) / n = th g2/5 * sinc(h) * (-sin h - i cos h),
  // h = th g2 n / 10: no division by n, so empty or denormal sites stay finite
  W.cs = cx<T>{-ang.tg25 * sinc * s2, -ang.tg25 * sinc * c2};

  // frame of F: u = e^{i alpha}, cos beta, sin beta.  With F_perp = 0, beta is 0 or pi
  // exactly, and d(beta) is taken exactly diagonal or anti-diagonal, so that components that
  // are zero and have no source stay exactly zero.
  const cx<T> u{has_perp ? Fx * ip : T(1), has_perp ? Fy * ip : T(0)};
  const T cz = Fz >= T(0) ? T(1) : T(-1), cp = Fz * iF;
  const T cf = has_perp ? cp : cz;
  const T cb = has_F ? cf : T(1);
  const T sb = Fperp * iF;   // 0 without F
  W.u = u;
  W.u2 = u * u;
  // spin-2 Wigner small-d matrix d(beta) in the blocks of d_apply
  W.d = d_blocks(cb, sb);
}

// x <- exp(-i th g0 n) R P x for one 5-vector x (a or b).
//
// Both factors only add small corrections to x: the singlet part sv = cs (v^H x) v
// and the rotation part Phi t.  In FP32 they are summed first and added to x once, so
// the full-magnitude value is rounded a single time per application; rounding it
// after each factor made the FP32 qubit norm drift systematically (6e-5 over
// 20000 steps of the 1D two-soliton run, against 9e-7 with one rounding).  In FP64
// that drift is some 1e9 times smaller, and y = x + sv is formed once, by five complex
// multiply-adds, as the rotation's input and the base its correction is added to:
// 20 instructions per vector fewer than forming sv, adding it to x, and adding it again.
template <typename T>
QLG_HD void w_apply(cx<T> (&x)[5], const WCoef<T>& W) {
  const cx<T> uc = conj(W.u), u2c = conj(W.u2);
  // singlet correction sv = cs (v^H x) v, conj(v_m) = (-1)^m psi_{-m}, v_m = (-1)^m conj(psi_{-m})
  cx<T> s = W.p[4] * x[0];
  s = cfma(T(-1) * W.p[3], x[1], s);
  s = cfma(W.p[2], x[2], s);
  s = cfma(T(-1) * W.p[1], x[3], s);
  s = cfma(W.p[0], x[4], s);
  const cx<T> tt = W.cs * s;
  if constexpr (sizeof(T) == 8) {
    cx<T> y[5];   // x + sv
    y[0] = cfma(tt, conj(W.p[4]), x[0]);
    y[1] = cfma(tt, T(-1) * conj(W.p[3]), x[1]);
    y[2] = cfma(tt, conj(W.p[2]), x[2]);
    y[3] = cfma(tt, T(-1) * conj(W.p[1]), x[3]);
    y[4] = cfma(tt, conj(W.p[0]), x[4]);
    // w = Phi^* y; z = (Lambda' - I) d^T w; t = d z; x = y + Phi t
    cx<T> w[5];
    w[0] = y[0] * W.u2;
    w[1] = y[1] * W.u;
    w[2] = y[2];
    w[3] = y[3] * uc;
    w[4] = y[4] * u2c;
    cx<T> z[5];
    d_apply<T, true>(W.d, w, z);
#pragma unroll
    for (int k = 0; k < 5; ++k) z[k] = W.dl[k] * z[k];
    cx<T> t5[5];
    d_apply<T, false>(W.d, z, t5);
    x[0] = cfma(t5[0], u2c, y[0]);
    x[1] = cfma(t5[1], uc, y[1]);
    x[2] = y[2] + t5[2];
    x[3] = cfma(t5[3], W.u, y[3]);
    x[4] = cfma(t5[4], W.u2, y[4]);
    return;
  }
  cx<T> sv[5];
  sv[0] = tt * conj(W.p[4]);
  sv[1] = tt * (T(-1) * conj(W.p[3]));
  sv[2] = tt * conj(W.p[2]);
  sv[3] = tt * (T(-1) * conj(W.p[1]));
  sv[4] = tt * conj(W.p[0]);
  // w = Phi^* (x + sv): input of the rotation's (small) correction
  cx<T> w[5];
  w[0] = (x[0] + sv[0]) * W.u2;
  w[1] = (x[1] + sv[1]) * W.u;
  w[2] = x[2] + sv[2];
  w[3] = (x[3] + sv[3]) * uc;
  w[4] = (x[4] + sv[4]) * u2c;
  // z = (Lambda' - I) d^T w
  cx<T> z[5];
  d_apply<T, true>(W.d, w, z);
#pragma unroll
  for (int k = 0; k < 5; ++k) z[k] = W.dl[k] * z[k];
  // t = d z; x += sv + Phi t
  cx<T> t5[5];
  d_apply<T, false>(W.d, z, t5);
  x[0] = x[0] + cfma(t5[0], u2c, sv[0]);
  x[1] = x[1] + cfma(t5[1], uc, sv[1]);
  x[2] = x[2] + (t5[2] + sv[2]);
  x[3] = x[3] + cfma(t5[3], W.u, sv[3]);
  x[4] = x[4] + cfma(t5[4], W.u2, sv[4]);
}

template <typename T, bool kExt = false>
QLG_HD void potential(cx<T> (&a)[5], cx<T> (&b)[5], const Angles<T> ang, T ext = T(0)) {
  WCoef<T> W;
  w_coefficients<T, kExt>(a, b, ang, W, ext);
  w_apply(a, W);
  w_apply(b, W);
}

}  // namespace qlg
