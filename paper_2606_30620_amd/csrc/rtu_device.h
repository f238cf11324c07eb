// Device math of the RTU-grid lens model for gfx950 (wave64).
//
// Lens deflections (App. A), their vector-Jacobian products with respect to the
// lens parameters, the Hermite CDF spline (App. C step iv), the softplus
// positivity transform (eqs. 2-3) and the radix-2 FFT used for the Gaussian
// process (eq. 1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtu_internal.h"

namespace rtu {

// Chebyshev nodes u_k on (0, 1) and the FP64 matrix D with p'(u_k) = sum_l D_kl q_l
// (derivative of the degree-21 interpolant through the quantiles q_l).
extern __constant__ float c_u[K];
extern __constant__ double c_D[K * K];
// exp(-2 pi i k / 256), k < 128
extern __constant__ float2 c_tw[128];

// ------------------------------------------------------------------ softplus
// log(1 + u) for u >= 0 without cancellation: log(w) u / (w - 1) with
// w = 1 + u rounded (Goldberg 1991, Theorem 4)
__device__ __forceinline__ float log1p_pos(float u) {
  const float w = 1.f + u;
  return w == 1.f ? u : __logf(w) * (u / (w - 1.f));
}
__device__ __forceinline__ float softplus_f(float x) {
  return fmaxf(x, 0.f) + log1p_pos(__expf(-fabsf(x)));
}
// log(softplus(x)), finite for all x
__device__ __forceinline__ float log_softplus_f(float x) {
  return x < -15.f ? x : __logf(softplus_f(x));
}
// softplus(x), log softplus(x) and sigmoid(x) / softplus(x) from one exponential
struct SoftplusTerms {
  float lsp, ratio;
};
__device__ __forceinline__ SoftplusTerms softplus_terms(float x) {
  const float e = __expf(-fabsf(x));                 // (0, 1]
  const float sp = fmaxf(x, 0.f) + log1p_pos(e);     // softplus(x)
  const float sig = (x >= 0.f ? 1.f : e) / (1.f + e);
  SoftplusTerms o;
  // below -15 both tend to e^x (which may underflow): the ratio is 1 - e^x/2
  o.lsp = x < -15.f ? x : __logf(sp);
  o.ratio = x < -15.f ? 1.f - 0.5f * e : sig / sp;
  return o;
}

// ------------------------------------------------------------------ SIE + shear
// Per-sample constants of the singular isothermal ellipsoid (eq. A1 at slope 2)
// kappa = (theta_E/2) / sqrt(q x'^2 + y'^2/q) and of the external shear.
// Below this |(e1, e2)| the gradient with respect to the lens parameters is
// formed without the position angle (sie_vjp_round): the angle is undefined at
// e = 0, and its derivative terms cancel to O(e) in FP32 near it.
constexpr float E_ROUND = 0.02f;

// (struct Sie: rtu_internal.h, where the per-sample copies live)

__device__ __forceinline__ Sie make_sie(const float* L) {
  Sie o;
  o.the = L[0]; o.e1 = L[1]; o.e2 = L[2]; o.x0 = L[3]; o.y0 = L[4]; o.g1 = L[5]; o.g2 = L[6];
  o.e = sqrtf(o.e1 * o.e1 + o.e2 * o.e2);
  o.q = (1.f - o.e) / (1.f + o.e);
  const float phi = 0.5f * atan2f(o.e2, o.e1);
  sincosf(phi, &o.s, &o.c);
  o.f = 2.f * sqrtf(o.e) / (1.f + o.e);   // sqrt(1 - q^2) without cancellation
  o.P = o.the * sqrtf(o.q);
  o.q2 = o.q * o.q;
  o.invf = o.f > 0.f ? 1.f / o.f : 0.f;
  o.round = o.e < E_ROUND;
  const float ie = 1.f / (1.f + o.e);
  o.cpe = o.c * ie; o.spe = o.s * ie;
  o.cq = o.c * o.q; o.sq = o.s * o.q;
  o.im2f = ie * ie;
  o.jb = fabsf(o.the) / sqrtf(o.q);
  o.gam = sqrtf(o.g1 * o.g1 + o.g2 * o.g2);
  return o;
}

// ------------------------------------------------------------------ fast math
// Hardware reciprocal, square root and base-2 logarithm (about 1 ulp each).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fln(float x) { return 0.69314718055994531f * __builtin_amdgcn_logf(x); }

// atan(x)/x = P(x^2) and atanh(x)/x = Q(x^2): least-squares fits made by
// csrc/gen_poly.py (max relative error of the FP32 evaluation 1.4e-7 on
// [0, 1] and 1.2e-7 on [0, 1/2]).
__device__ __forceinline__ float poly_atan(float t) {
  float p = 0.0028340642f;
  p = fmaf(p, t, -0.01600503f); p = fmaf(p, t, 0.042587608f); p = fmaf(p, t, -0.07495446f);
  p = fmaf(p, t, 0.10636754f);  p = fmaf(p, t, -0.14202571f); p = fmaf(p, t, 0.19992484f);
  p = fmaf(p, t, -0.33333066f); p = fmaf(p, t, 1.0f);
  return p;
}
__device__ __forceinline__ float poly_atan_d(float t) {   // d P / d t
  float p = 8.f * 0.0028340642f;
  p = fmaf(p, t, 7.f * -0.01600503f); p = fmaf(p, t, 6.f * 0.042587608f); p = fmaf(p, t, 5.f * -0.07495446f);
  p = fmaf(p, t, 4.f * 0.10636754f);  p = fmaf(p, t, 3.f * -0.14202571f); p = fmaf(p, t, 2.f * 0.19992484f);
  p = fmaf(p, t, -0.33333066f);
  return p;
}
__device__ __forceinline__ float poly_atanh(float t) {
  float p = 0.1783732f;
  p = fmaf(p, t, 0.04998629f); p = fmaf(p, t, 0.11866759f); p = fmaf(p, t, 0.14216292f);
  p = fmaf(p, t, 0.2000299f);  p = fmaf(p, t, 0.33333287f); p = fmaf(p, t, 1.0f);
  return p;
}
__device__ __forceinline__ float poly_atanh_d(float t) {
  float p = 6.f * 0.1783732f;
  p = fmaf(p, t, 5.f * 0.04998629f); p = fmaf(p, t, 4.f * 0.11866759f); p = fmaf(p, t, 3.f * 0.14216292f);
  p = fmaf(p, t, 2.f * 0.2000299f);  p = fmaf(p, t, 0.33333287f);
  return p;
}

// atan(f a)/f and, with D, its derivative 1/(1 + (f a)^2) in a: the polynomial
// in (f a)^2 for |f a| <= 1, else pi/2 - atan(1/|f a|) with the same
// polynomial.  The second form is evaluated only when a lane of the wave
// needs it (a wave-uniform branch), and then selected per lane.  The
// derivative in f is (a da - v)/f; the vector-Jacobian product forms it from
// these two (sie_shear_vjp), so it needs no polynomial of its own.
template <bool D>
__device__ __forceinline__ void atan_over_f(float f, float invf, float a, float& v, float& da) {
  const float fa = f * a, t = fa * fa;
  const bool big = t > 1.f;
  const bool any_big = __any(big);
  float r = 0.f, arg = t;
  if (any_big) {
    r = rcp(fabsf(fa));
    arg = big ? r * r : t;
  }
  const float p = poly_atan(arg);
  v = a * p;
  if (D) da = rcp(1.f + t);
  if (any_big) {
    const float vb = copysignf(1.5707963267948966f - r * p, fa) * invf;
    v = big ? vb : v;
  }
}
// atanh(f b)/f and, with D, its derivative 1/(1 - (f b)^2) in b (|f b| < 1):
// the polynomial in (f b)^2 for (f b)^2 <= 1/4, else the logarithm, evaluated
// when a lane of the wave needs it.
template <bool D>
__device__ __forceinline__ void atanh_over_f(float f, float invf, float b, float& v, float& db) {
  const float fb = f * b, t = fb * fb;
  const bool big = t > 0.25f;
  v = b * poly_atanh(t);
  if (D) db = rcp(1.f - t);
  if (__any(big)) {
    const float vl = 0.5f * fln((1.f + fb) * rcp(1.f - fb)) * invf;
    v = big ? vl : v;
  }
}

// Per-ray intermediates of the SIE deflection, kept for the VJP.
struct SieRay {
  float xp, yp, ip, a, b, A, dA, B, dB;
  bool ok;
};

// Deflection of SIE + shear at (x, y); with D the partial derivatives needed by
// sie_shear_vjp are kept in E.
template <bool D>
__device__ __forceinline__ void sie_shear_alpha(const Sie& L, float x, float y, float& ax, float& ay,
                                                SieRay& E) {
  const float dx = x - L.x0, dy = y - L.y0;
  E.xp = L.c * dx + L.s * dy;
  E.yp = -L.s * dx + L.c * dy;
  const float qx = L.q * E.xp;
  const float psi2 = qx * qx + E.yp * E.yp;
  // a ray at the lens centre (psi = 0) is not deflected by the SIE; it takes
  // the same arithmetic on a clamped psi and its result is selected away
  E.ok = psi2 > 1e-30f;
  E.ip = __builtin_amdgcn_rsqf(fmaxf(psi2, 1e-30f));
  E.a = E.xp * E.ip;
  E.b = E.yp * E.ip;
  atan_over_f<D>(L.f, L.invf, E.a, E.A, E.dA);
  atanh_over_f<D>(L.f, L.invf, E.b, E.B, E.dB);
  const float axp = E.ok ? L.P * E.A : 0.f;
  const float ayp = E.ok ? L.P * E.B : 0.f;
  ax = L.c * axp - L.s * ayp + L.g1 * x + L.g2 * y;
  ay = L.s * axp + L.c * ayp + L.g2 * x - L.g1 * y;
}

__device__ __forceinline__ void sie_shear_alpha(const Sie& L, float x, float y, float& ax, float& ay) {
  SieRay E;
  sie_shear_alpha<false>(L, x, y, ax, ay, E);
}

// Accumulators of the SIE + shear vector-Jacobian product, summed over rays
// and converted to parameter gradients once per sample by sie_grad_one().
// Every factor that is constant per sample (P, q, 1/f, the rotation back to
// the sky frame) is left to that conversion, so a ray adds only its own terms.
// With abar' = R(-phi) abar the loss gradient in the lens frame, per ray:
//   P   += abar'_x A + abar'_y B                    (d loss/d P)
//   q   += psi' x' a,  psi' = -(a' a + b' b)/psi   (d loss/d q through psi, / (P q))
//          with a' = abar'_x dA, b' = abar'_y dB
//   f   += (a' a + b' b) - (abar'_x A + abar'_y B)  (d loss/d f, / (P/f): the
//          derivative of atan(f a)/f in f is (a dA - A)/f, likewise for atanh)
//   phi += abar'_y A - abar'_x B + x'' y' - y'' x'  (d loss/d phi, / P)
//   x0, y0 += x'', y'',  x'' = (a' + psi' q^2 x')/psi, y'' = (b' + psi' y')/psi
//          (d loss/d (x0, y0) = -P R(phi) (x0, y0) sums)
//   g1, g2: the shear gradient itself.
// A nearly round lens (sie_vjp_round) fills the same slots with the terms of
// its own chain.
struct SieAcc {
  float P, q, f, phi, x0, y0, g1, g2;
  __device__ __forceinline__ void zero() { P = q = f = phi = x0 = y0 = g1 = g2 = 0.f; }
};

// The SIE part of the vector-Jacobian product for a nearly round lens, with
// no position angle.  In complex notation (z = (x - x0) + i (y - y0), eps =
// e1 + i e2, abar = d loss/d alpha_x + i d loss/d alpha_y) the deflection is
//   alpha = K u G(w),  K = theta_E sqrt(1 - e^2),  m = z - eps conj(z),
//   u = m/|m|,  w = conj(eps) u^2,  G(w) = atan(sqrt w)/sqrt w
// (the elliptical power law in the hypergeometric form of Tessore & Metcalf
// 2015 at slope 2).  Since |u| = 1, du = i u Im(dm/m), and
//   d(u G) = tau_r Im(dm/m) + u^3 G'(w) d conj(eps),  tau_r = i u (G + 2 w G'),
// with dm = -conj(z) d eps - d z0 + eps d conj(z0).  Per ray this adds, without
// the factor K (applied once per sample by sie_grad_one):
//   P <- Re(conj(abar) H), H = u G (so d loss/d theta_E = sqrt(1-e^2) P),
//   q <- d/d e1, f <- d/d e2, x0, y0 <- d/d x0, y0 (phi stays 0).
// u G is the closed-form deflection already computed (E.A, E.B rotated back,
// divided by K), u = R(phi) (q a, b); |m| = psi (1 + e); G' is the series
// sum_{k>=1} (-1)^k k w^(k-1)/(2k+1), |w| = e < E_ROUND (five terms: 2e-9).
__device__ __forceinline__ void sie_vjp_round(const Sie& L, const SieRay& E, float x, float y, float abx,
                                              float aby, SieAcc& acc) {
  const float Hx = L.cpe * E.A - L.spe * E.B, Hy = L.spe * E.A + L.cpe * E.B;
  const float ux = L.cq * E.a - L.s * E.b, uy = L.sq * E.a + L.c * E.b;
  const float u2x = ux * ux - uy * uy, u2y = 2.f * ux * uy;
  const float wx = L.e1 * u2x + L.e2 * u2y, wy = L.e1 * u2y - L.e2 * u2x;
  const float Gx = Hx * ux + Hy * uy, Gy = Hy * ux - Hx * uy;        // H conj(u)
  float px = -5.f / 11.f, py = 0.f;                                  // G'(w), Horner
  {
    constexpr float cf[4] = {4.f / 9.f, -3.f / 7.f, 2.f / 5.f, -1.f / 3.f};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float tx = px * wx - py * wy + cf[k], ty = px * wy + py * wx;
      px = tx; py = ty;
    }
  }
  const float g2x = Gx + 2.f * (wx * px - wy * py), g2y = Gy + 2.f * (wx * py + wy * px);
  const float ugx = ux * g2x - uy * g2y, ugy = ux * g2y + uy * g2x;
  const float tau = -abx * ugy + aby * ugx;                          // Re(conj(abar) i u g2)
  const float u3x = u2x * ux - u2y * uy, u3y = u2x * uy + u2y * ux;
  const float sx = u3x * px - u3y * py, sy = u3x * py + u3y * px;    // u^3 G'
  const float sgx = abx * sx + aby * sy, sgy = abx * sy - aby * sx;  // conj(abar) u^3 G'
  const float dx = x - L.x0, dy = y - L.y0;
  const float mx = (1.f - L.e1) * dx - L.e2 * dy, my = (1.f + L.e1) * dy - L.e2 * dx;
  const float im2 = E.ip * E.ip * L.im2f;                            // 1/|m|^2
  const float zmx = dx * mx - dy * my, zmy = dx * my + dy * mx;       // z m
  const float zbmx = zmx * im2, zbmy = -zmy * im2;                    // conj(z)/m
  const float imx = mx * im2, imy = -my * im2;                        // 1/m
  const float emx = (L.e1 * mx + L.e2 * my) * im2, emy = (L.e2 * mx - L.e1 * my) * im2;   // eps/m
  acc.P += abx * Hx + aby * Hy;
  acc.q += sgx - tau * zbmy;
  acc.f += sgy - tau * zbmx;
  acc.x0 += tau * (emy - imy);
  acc.y0 -= tau * (imx + emx);
}

// Given d loss / d alpha at (x, y) and the ray's SIE intermediates, accumulate
// d loss / d (internal SIE quantities) and the shear gradient.
__device__ __forceinline__ void sie_shear_vjp(const Sie& L, const SieRay& E, float x, float y, float abx,
                                              float aby, SieAcc& acc) {
  acc.g1 += abx * x - aby * y;
  acc.g2 += abx * y + aby * x;
  // the SIE part contributes nothing for a ray at the lens centre
  const float m = E.ok ? 1.f : 0.f;
  abx *= m;
  aby *= m;
  if (L.round) {   // one lens per workgroup: uniform
    sie_vjp_round(L, E, x, y, abx, aby, acc);
    return;
  }
  const float axpb = L.c * abx + L.s * aby;          // abar in the lens frame
  const float aypb = -L.s * abx + L.c * aby;
  const float pterm = axpb * E.A + aypb * E.B;
  const float ab = axpb * E.dA, bb = aypb * E.dB;
  const float sab = ab * E.a + bb * E.b;
  const float psib = -sab * E.ip;
  const float t1 = psib * E.xp;
  const float xpb = fmaf(t1, L.q2, ab) * E.ip;
  const float ypb = fmaf(psib, E.yp, bb) * E.ip;
  acc.P += pterm;
  acc.q = fmaf(t1, E.a, acc.q);
  acc.f += sab - pterm;
  acc.phi += (aypb * E.A - axpb * E.B) + (xpb * E.yp - ypb * E.xp);
  acc.x0 += xpb;
  acc.y0 += ypb;
}

// Component k < 7 of d loss / d (theta_E, e1, e2, x0, y0, g1, g2) from the
// summed accumulators a (see SieAcc): the per-sample factors, then the chain
// (P, q, f, phi) -> (theta_E, e) -> (e1, e2).  A nearly round lens summed the
// angle-free terms of sie_vjp_round: theta_E enters through K = theta_E
// sqrt(1 - e^2) alone.
__device__ __forceinline__ double sie_grad_one(const Sie& L, const double* a, int k) {
  if (L.round) {
    const double ee = (double)L.e1 * L.e1 + (double)L.e2 * L.e2, r = sqrt(1.0 - ee);
    const double K = (double)L.the * r;
    switch (k) {
      case 0: return a[0] * r;
      case 1: return K * a[1] - a[0] * (double)L.the * (double)L.e1 / r;
      case 2: return K * a[2] - a[0] * (double)L.the * (double)L.e2 / r;
      case 3: return K * a[4];
      case 4: return K * a[5];
      default: return a[k + 1];
    }
  }
  const double q = L.q, sq = sqrt(q), e = (double)L.e, P = (double)L.the * sq;
  const double c = L.c, s = L.s;
  switch (k) {
    case 0: return a[0] * sq;
    case 3: return -P * (c * a[4] - s * a[5]);
    case 4: return -P * (s * a[4] + c * a[5]);
    case 5: return a[6];
    case 6: return a[7];
    default: break;
  }
  // d loss/d q (through psi and through P), d loss/d f, d loss/d phi
  const double qb = P * q * a[1] + a[0] * (double)L.the / (2.0 * sq);
  const double fb = P / (double)L.f * a[2];
  const double phib = P * a[3];
  const double dqde = -2.0 / ((1.0 + e) * (1.0 + e));
  const double dfde = (1.0 - e) / (sqrt(e) * (1.0 + e) * (1.0 + e));
  const double eb = qb * dqde + fb * dfde;
  const double e1 = L.e1, e2 = L.e2;
  return k == 1 ? eb * e1 / e - phib * e2 / (2.0 * e * e) : eb * e2 / e + phib * e1 / (2.0 * e * e);
}
__device__ __forceinline__ void sie_grad(const Sie& L, const double* a, double* g) {
  for (int k = 0; k < 7; ++k) g[k] = sie_grad_one(L, a, k);
}

// ------------------------------------------------------------------ EPL (App. A.1)
// Elliptical power law, kappa = (3 - gamma)/2 (theta_E/rho)^(gamma - 1), in
// the angle-free complex form of the Tessore & Metcalf (2015) deflection: with
// z = (x - x0) + i (y - y0), eps = e1 + i e2, m = z - eps conj(z), u = m/|m|,
// t = gamma - 1 and Lam = theta_E sqrt(1 - |eps|^2),
//   alpha = Lam^t |m|^(-t) m F(w),  w = -conj(eps) u^2,
//   F(w) = 2F1(1, t/2; 2 - t/2; w) = sum_n c_n w^n,  c_n = c_{n-1} (2n-2+t)/(2n+2-t),
// summed by Horner's rule over the terms that reach FP32 precision (|w| =
// |eps|).  It has no angle, so the gradient is smooth at eps = 0.
constexpr int EPL_NMAX = 48;             // series terms at most (|eps| <= 0.68 reaches 1e-8)

struct Epl {
  float the, e1, e2, x0, y0, g1, g2, t;
  float l2lam;     // log2 Lam
  float hk;        // 1 / (2 (1 - |eps|^2))
};
// Per-sample coefficient tables: c_n (F), (n+1) c_{n+1} (F' = dF/dw) and
// c_n s_n with s_n = d ln c_n / dt = sum_{k<=n} 1/(2k-2+t) + 1/(2k+2-t) (dF/dt).
struct EplTab {
  float c[EPL_NMAX], cd[EPL_NMAX], cs[EPL_NMAX];
  int n;
};

__device__ __forceinline__ Epl make_epl(const float* L) {
  Epl o;
  o.the = L[0]; o.e1 = L[1]; o.e2 = L[2]; o.x0 = L[3]; o.y0 = L[4]; o.g1 = L[5]; o.g2 = L[6];
  o.t = L[7] - 1.f;
  const float omee = 1.f - (o.e1 * o.e1 + o.e2 * o.e2);
  o.l2lam = log2f(o.the * sqrtf(omee));
  o.hk = 0.5f / omee;
  return o;
}

// The tables of one sample, by one thread (FP64, stored FP32).
__device__ __forceinline__ void epl_table(const Epl& E, EplTab& T) {
  const double t = E.t, e = sqrt((double)E.e1 * E.e1 + (double)E.e2 * E.e2);
  double c = 1.0, sn = 0.0, en = 1.0;
  int n = 0;
  for (; n < EPL_NMAX; ++n) {
    T.c[n] = (float)c;
    T.cs[n] = (float)(c * sn);
    if (n > 0) T.cd[n - 1] = (float)(n * c);
    if (n > 0 && c * en < 1e-9) { ++n; break; }
    const double a = 2.0 * n + t, bb = 2.0 * n + 4.0 - t;   // (2k-2+t), (2k+2-t) at k = n+1
    c *= a / bb;
    sn += 1.0 / a + 1.0 / bb;
    en *= e;
  }
  T.n = n;
  T.cd[n - 1] = 0.f;
}

// The per-ray quantities shared by the deflection and its vector-Jacobian
// product.
struct EplRay {
  float dx, dy, mr, mi, ir, u2r, u2i, wr, wi, pw, Fr, Fi;
  bool ok;
};
__device__ __forceinline__ void epl_ray(const Epl& L, const EplTab& T, float x, float y, EplRay& R) {
  R.dx = x - L.x0; R.dy = y - L.y0;
  R.mr = R.dx - (L.e1 * R.dx + L.e2 * R.dy);
  R.mi = R.dy - (L.e2 * R.dx - L.e1 * R.dy);
  const float r2 = R.mr * R.mr + R.mi * R.mi;
  R.ok = r2 > 0.f;
  R.ir = __builtin_amdgcn_rsqf(fmaxf(r2, 1e-30f));
  const float ur = R.mr * R.ir, ui = R.mi * R.ir;
  R.u2r = ur * ur - ui * ui;
  R.u2i = 2.f * ur * ui;
  R.wr = -(L.e1 * R.u2r + L.e2 * R.u2i);
  R.wi = -(L.e1 * R.u2i - L.e2 * R.u2r);
  // Lam^t |m|^-t
  R.pw = exp2f(L.t * (L.l2lam + log2f(R.ir)));
  float Fr = T.c[T.n - 1], Fi = 0.f;
  for (int k = T.n - 2; k >= 0; --k) {
    const float nr = fmaf(Fr, R.wr, fmaf(-Fi, R.wi, T.c[k]));
    Fi = fmaf(Fr, R.wi, Fi * R.wr);
    Fr = nr;
  }
  R.Fr = Fr; R.Fi = Fi;
}

__device__ __forceinline__ void epl_shear_alpha(const Epl& L, const EplTab& T, float x, float y, float& ax,
                                                float& ay) {
  EplRay R;
  epl_ray(L, T, x, y, R);
  const float s = R.ok ? R.pw : 0.f;
  ax = s * (R.mr * R.Fr - R.mi * R.Fi) + L.g1 * x + L.g2 * y;
  ay = s * (R.mr * R.Fi + R.mi * R.Fr) + L.g2 * x - L.g1 * y;
}

// Vector-Jacobian product of EPL + shear: given gbar = d loss/d alpha, adds
// d loss/d (theta_E, e1, e2, x0, y0, gamma1, gamma2, gamma) to acc.  With
// Wirtinger derivatives (alpha = Lam^t m^(1-t/2) conj(m)^(-t/2) F(-conj(eps) m/conj(m))):
//   d alpha/d m       = pw [(1 - t/2) F - F' conj(eps) u^2]
//   d alpha/d conj(m) = pw [-(t/2) F u^2 + F' conj(eps) u^4]
//   d alpha/d conj(eps) at fixed m adds -pw m F' u^2, and through Lam
//   d alpha/d eps = -t alpha conj(eps) / (2 (1 - |eps|^2)) (conjugate for conj(eps));
// m = Delta - eps conj(Delta) with Delta = z - z0 carries them to z0 and eps,
// and a real pair (p_x, p_y) of a complex parameter p gets
//   d loss/d p_x = Re(conj(gbar) (D_p + D_conj(p))),  d loss/d p_y = -Im(conj(gbar) (D_p - D_conj(p))).
__device__ __forceinline__ void epl_shear_vjp(const Epl& L, const EplTab& T, float x, float y, float gx,
                                              float gy, float (&acc)[8]) {
  EplRay R;
  R.dx = x - L.x0; R.dy = y - L.y0;
  R.mr = R.dx - (L.e1 * R.dx + L.e2 * R.dy);
  R.mi = R.dy - (L.e2 * R.dx - L.e1 * R.dy);
  const float r2 = R.mr * R.mr + R.mi * R.mi;
  acc[5] += gx * x - gy * y;
  acc[6] += gx * y + gy * x;
  if (!(r2 > 0.f)) return;
  R.ir = __builtin_amdgcn_rsqf(r2);
  const float ur = R.mr * R.ir, ui = R.mi * R.ir;
  R.u2r = ur * ur - ui * ui;
  R.u2i = 2.f * ur * ui;
  R.wr = -(L.e1 * R.u2r + L.e2 * R.u2i);
  R.wi = -(L.e1 * R.u2i - L.e2 * R.u2r);
  const float l2 = L.l2lam + log2f(R.ir);      // log2(Lam/|m|)
  const float pw = exp2f(L.t * l2);
  // F, F' and dF/dt by Horner's rule
  float Fr = T.c[T.n - 1], Fi = 0.f, Dr = T.cd[T.n - 1], Di = 0.f, Sr = T.cs[T.n - 1], Si = 0.f;
  for (int k = T.n - 2; k >= 0; --k) {
    float nr = fmaf(Fr, R.wr, fmaf(-Fi, R.wi, T.c[k]));
    Fi = fmaf(Fr, R.wi, Fi * R.wr);
    Fr = nr;
    nr = fmaf(Dr, R.wr, fmaf(-Di, R.wi, T.cd[k]));
    Di = fmaf(Dr, R.wi, Di * R.wr);
    Dr = nr;
    nr = fmaf(Sr, R.wr, fmaf(-Si, R.wi, T.cs[k]));
    Si = fmaf(Sr, R.wi, Si * R.wr);
    Sr = nr;
  }
  const float t = L.t;
  // alpha = pw m F;  A = pw m
  const float Ar = pw * R.mr, Ai = pw * R.mi;
  const float alr = Ar * Fr - Ai * Fi, ali = Ar * Fi + Ai * Fr;
  // E = conj(eps) u^2 (complex), F' E, F' E u^2
  const float Er = L.e1 * R.u2r + L.e2 * R.u2i, Ei = L.e1 * R.u2i - L.e2 * R.u2r;
  const float DEr = Dr * Er - Di * Ei, DEi = Dr * Ei + Di * Er;
  const float DE2r = DEr * R.u2r - DEi * R.u2i, DE2i = DEr * R.u2i + DEi * R.u2r;
  const float FU2r = Fr * R.u2r - Fi * R.u2i, FU2i = Fr * R.u2i + Fi * R.u2r;
  // P1 = d alpha/d m, P2 = d alpha/d conj(m)
  const float P1r = pw * ((1.f - 0.5f * t) * Fr - DEr), P1i = pw * ((1.f - 0.5f * t) * Fi - DEi);
  const float P2r = pw * (-0.5f * t * FU2r + DE2r), P2i = pw * (-0.5f * t * FU2i + DE2i);
  // z0: D = -P1 + conj(eps) P2,  Db = eps P1 - P2
  const float Dz_r = -P1r + (L.e1 * P2r + L.e2 * P2i), Dz_i = -P1i + (L.e1 * P2i - L.e2 * P2r);
  const float Dzb_r = (L.e1 * P1r - L.e2 * P1i) - P2r, Dzb_i = (L.e1 * P1i + L.e2 * P1r) - P2i;
  // eps: D = -conj(Delta) P1 - t hk alpha conj(eps)
  //      Db = -Delta P2 - pw m F' u^2 - t hk alpha eps
  const float th = t * L.hk;
  const float De_r = -(R.dx * P1r + R.dy * P1i) - th * (alr * L.e1 + ali * L.e2);
  const float De_i = -(R.dx * P1i - R.dy * P1r) - th * (ali * L.e1 - alr * L.e2);
  const float Du2r = Dr * R.u2r - Di * R.u2i, Du2i = Dr * R.u2i + Di * R.u2r;   // F' u^2
  const float Deb_r = -(R.dx * P2r - R.dy * P2i) - (Ar * Du2r - Ai * Du2i) - th * (alr * L.e1 - ali * L.e2);
  const float Deb_i = -(R.dx * P2i + R.dy * P2r) - (Ar * Du2i + Ai * Du2r) - th * (ali * L.e1 + alr * L.e2);
  // Re(conj(g) X) = gx Xr + gy Xi;  Im(conj(g) X) = gx Xi - gy Xr
  acc[0] += L.the > 0.f ? t * (gx * alr + gy * ali) / L.the : 0.f;
  acc[1] += gx * (De_r + Deb_r) + gy * (De_i + Deb_i);
  acc[2] += -(gx * (De_i - Deb_i) - gy * (De_r - Deb_r));
  acc[3] += gx * (Dz_r + Dzb_r) + gy * (Dz_i + Dzb_i);
  acc[4] += -(gx * (Dz_i - Dzb_i) - gy * (Dz_r - Dzb_r));
  // gamma: alpha ln(Lam/|m|) + A dF/dt
  const float ln = 0.69314718f * l2;
  const float Tr = alr * ln + (Ar * Sr - Ai * Si), Ti = ali * ln + (Ar * Si + Ai * Sr);
  acc[7] += gx * Tr + gy * Ti;
}

// ------------------------------------------------------------------ NFW (App. A.2)
// T(v) = atanh(sqrt v)/sqrt v (v > 0), atan(sqrt(-v))/sqrt(-v) (v < 0), 1 at 0:
// Q(v) and P(-v) of the polynomials above where they apply.
__device__ __forceinline__ float nfw_T(float v) {
  if (v >= 0.f) {
    if (v <= 0.25f) return poly_atanh(v);
    const float sq = fsqrt(v);
    return 0.5f * fln((1.f + sq) * rcp(1.f - sq)) * rcp(sq);
  }
  if (v >= -1.f) return poly_atan(-v);
  const float sq = fsqrt(-v), r = rcp(sq);
  return (1.5707963267948966f - r * poly_atan(r * r)) * r;
}

// Projected-mass function h(X) of the NFW convergence (eq. A3) and h'(X) = X G(X),
// G = (1 - F(X))/(X^2 - 1) = kappa/(2 kappa_s).
__device__ __forceinline__ void nfw_h_dh(float X, float& h, float& dh) {
  if (X < 1e-6f) {
    const float L = fln(2.f * rcp(X));
    h = X * X * (0.5f * L - 0.25f);
    dh = X * (L - 1.f);
    return;
  }
  if (X < 0.5f) {
    // c = sqrt(1 - X^2); 2 atanh(sqrt((1-X)/(1+X))) = ln((1+c)/X)
    const float X2 = X * X;
    const float c = fsqrt(1.f - X2), ic = rcp(c), i1c = rcp(1.f + c);
    h = fln(2.f * rcp(X)) * X2 * i1c * ic + log1pf(-0.5f * X2 * i1c) * ic;
    const float F = 0.5f * fln((1.f + c) * (1.f + c) * rcp(X2)) * ic;   // atanh(c)/c
    dh = X * (F - 1.f) * ic * ic;
    return;
  }
  // F = atanh(sqrt(1 - X^2))/sqrt(1 - X^2) (atan beyond X = 1) = T(1 - X^2)
  // equals 2 T(v)/(1 + X), v = (1 - X)/(1 + X): with c = sqrt(1 - X^2),
  // atanh(c) = ln((1 + c)/X) = 2 atanh(sqrt v), and sqrt(v)/c = 1/(1 + X)
  const float ix1 = rcp(1.f + X);
  const float v = (1.f - X) * ix1;
  const float F = 2.f * nfw_T(v) * ix1;
  h = fln(0.5f * X) + F;
  const float vp = (1.f - X) * (1.f + X);
  float G;
  if (fabsf(vp) < 0.2f) {
    float r = 1.f / 25.f;
    r = fmaf(r, vp, 1.f / 23.f); r = fmaf(r, vp, 1.f / 21.f); r = fmaf(r, vp, 1.f / 19.f);
    r = fmaf(r, vp, 1.f / 17.f); r = fmaf(r, vp, 1.f / 15.f); r = fmaf(r, vp, 1.f / 13.f);
    r = fmaf(r, vp, 1.f / 11.f); r = fmaf(r, vp, 1.f / 9.f);  r = fmaf(r, vp, 1.f / 7.f);
    r = fmaf(r, vp, 1.f / 5.f);  r = fmaf(r, vp, 1.f / 3.f);
    G = r;
  } else {
    G = (F - 1.f) * rcp(vp);
  }
  dh = X * G;
}

struct Nfw {
  float ks, rs, xs, ys, irs, htau;  // htau = h(tau) (tau > 0)
};

__device__ __forceinline__ Nfw make_nfw(const float* p, float tau) {
  Nfw o;
  o.ks = p[0]; o.rs = p[1]; o.xs = p[2]; o.ys = p[3];
  o.irs = 1.f / o.rs;
  o.htau = 0.f;
  if (tau > 0.f) { float d; nfw_h_dh(tau, o.htau, d); }
  return o;
}

// alpha = 4 ks rs^2 H(X) d / r^2, d = theta - centre, X = r/rs, H = h(min(X, tau)).
__device__ __forceinline__ void nfw_alpha(const Nfw& N, float tau, float x, float y, float& ax, float& ay) {
  const float dx = x - N.xs, dy = y - N.ys;
  const float r2 = dx * dx + dy * dy;
  if (!(r2 > 1e-30f)) return;
  const float ir2 = rcp(r2);
  const float X = fsqrt(r2) * N.irs;
  float H, dH;
  if (tau > 0.f && X > tau) { H = N.htau; } else { nfw_h_dh(X, H, dH); }
  const float C = 4.f * N.ks * N.rs * N.rs * H * ir2;
  ax += C * dx;
  ay += C * dy;
}

// d loss/d(ks, rs, xs, ys) given d loss / d alpha.
__device__ __forceinline__ void nfw_vjp(const Nfw& N, float tau, float x, float y, float abx, float aby,
                                        float& gks, float& grs, float& gxs, float& gys) {
  const float dx = x - N.xs, dy = y - N.ys;
  const float r2 = dx * dx + dy * dy;
  if (!(r2 > 1e-30f)) return;
  const float r = fsqrt(r2), ir = rcp(r), ir2 = ir * ir;
  const float X = r * N.irs;
  float H, dH;
  if (tau > 0.f && X > tau) { H = N.htau; dH = 0.f; } else { nfw_h_dh(X, H, dH); }
  const float Y = abx * dx + aby * dy;
  const float rs = N.rs;
  gks += 4.f * rs * rs * H * Y * ir2;
  grs += Y * 4.f * N.ks * (2.f * rs * H - r * dH) * ir2;
  const float C = 4.f * N.ks * rs * rs * H * ir2;
  // C'(r)/r = 4 ks (rs H'/r^3 - 2 rs^2 H / r^4)
  const float Cpr = 4.f * N.ks * (rs * dH * ir - 2.f * rs * rs * H * ir2) * ir2;
  gxs -= C * abx + Y * Cpr * dx;
  gys -= C * aby + Y * Cpr * dy;
}

// nfw_alpha that also keeps what nfw_vjp needs at the same point: r (or -1
// where the deflection is skipped), h and h' (0 beyond the truncation), with
// the arithmetic of both, so that the adjoint evaluates h once per sub-ray.
__device__ __forceinline__ void nfw_alpha_keep(const Nfw& N, float tau, float x, float y, float& ax, float& ay,
                                               float& r, float& H, float& dH) {
  const float dx = x - N.xs, dy = y - N.ys;
  const float r2 = dx * dx + dy * dy;
  r = -1.f; H = 0.f; dH = 0.f;
  if (!(r2 > 1e-30f)) return;
  const float ir2 = rcp(r2);
  r = fsqrt(r2);
  const float X = r * N.irs;
  if (tau > 0.f && X > tau) { H = N.htau; dH = 0.f; } else { nfw_h_dh(X, H, dH); }
  const float C = 4.f * N.ks * N.rs * N.rs * H * ir2;
  ax += C * dx;
  ay += C * dy;
}
// nfw_vjp from the values nfw_alpha_keep kept.
__device__ __forceinline__ void nfw_vjp_kept(const Nfw& N, float x, float y, float abx, float aby, float r, float H,
                                             float dH, float& gks, float& grs, float& gxs, float& gys) {
  if (!(r > 0.f)) return;
  const float dx = x - N.xs, dy = y - N.ys;
  const float ir = rcp(r), ir2 = ir * ir;
  const float Y = abx * dx + aby * dy;
  const float rs = N.rs;
  gks += 4.f * rs * rs * H * Y * ir2;
  grs += Y * 4.f * N.ks * (2.f * rs * H - r * dH) * ir2;
  const float C = 4.f * N.ks * rs * rs * H * ir2;
  const float Cpr = 4.f * N.ks * (rs * dH * ir - 2.f * rs * rs * H * ir2) * ir2;
  gxs -= C * abx + Y * Cpr * dx;
  gys -= C * aby + Y * Cpr * dy;
}

// ------------------------------------------------------------------ CDF spline
// Number of knots <= z (0..K): the spline interval of z.
// Knot adjoint of one axis, accumulated per interval as moments
// m_j = sum ybar t^j of the rays in it; kb_flush turns them into
// d loss / d X_l, X_{l+1}, S_l, S_{l+1} (every partial derivative of the
// Hermite form is a cubic in t with interval-constant coefficients).
struct KnotMom {
  int k;
  float m0, m1, m2, m3;
};
__device__ __forceinline__ void km_add(KnotMom& c, float yb, float t) {
  const float yt = yb * t, yt2 = yt * t;
  c.m0 += yb; c.m1 += yt; c.m2 += yt2; c.m3 = fmaf(yt2, t, c.m3);
}
// The moments are linear in ybar, and so is the knot adjoint in them: a
// lane adds its moments to the tile's sums of interval k (km, FP64 in LDS)
// when it leaves the interval, and the knot adjoint is formed once per
// interval from the tile's sums (km_knots).
__device__ __forceinline__ void km_flush(KnotMom& c, double* km /* [K + 1][4] */) {
  if (c.k < 0) return;
  double* m = km + 4 * c.k;
  atomicAdd(&m[0], (double)c.m0);
  atomicAdd(&m[1], (double)c.m1);
  atomicAdd(&m[2], (double)c.m2);
  atomicAdd(&m[3], (double)c.m3);
  c.m0 = c.m1 = c.m2 = c.m3 = 0.f;
}
// d loss / d (X_l, X_r, S_l, S_r) of interval k from its moment sums m
// (l = k - 1, r = k for a Hermite interval; the linear continuations,
// interval 0: g = u_0 + S_0 (z - X_0) and interval K: the same at X_{K-1},
// depend on X_l and S_l only, with l = 0 and K - 1).  du[l] = u_{l+1} - u_l.
__device__ __forceinline__ void km_knots(int k, const double* m, const float* X, const float* S, const float* ih,
                                         const float* du_tab, double v[4]) {
  if (k == 0 || k >= K) {
    const int l = k == 0 ? 0 : K - 1;
    v[0] = -(double)S[l] * m[0]; v[1] = 0.0; v[2] = m[1]; v[3] = 0.0;
    return;
  }
  const int l = k - 1, r = k;
  const double h = (double)X[r] - (double)X[l], ihh = ih[l], Sl = S[l], Sr = S[r], du = du_tab[l];
  const double G10 = m[3] - 2.0 * m[2] + m[1];     // sum ybar (t^3 - 2t^2 + t)
  const double G11 = m[3] - m[2];                  // sum ybar (t^3 - t^2)
  const double gh = Sl * G10 + Sr * G11;           // sum ybar dg/dh at fixed t
  const double a0 = h * Sl, a1 = 6.0 * du - 4.0 * h * Sl - 2.0 * h * Sr, a2 = -6.0 * du + 3.0 * h * (Sl + Sr);
  const double Atm1 = -a0 * m[0] + (a0 - a1) * m[1] + (a1 - a2) * m[2] + a2 * m[3];  // sum ybar dg/dt (t-1)
  const double At = a0 * m[1] + a1 * m[2] + a2 * m[3];                              // sum ybar dg/dt t
  v[0] = Atm1 * ihh - gh;
  v[1] = gh - At * ihh;
  v[2] = h * G10;
  v[3] = h * G11;
}

// ------------------------------------------------------------------ lens light
// A lens-light Gaussian (App. A, Multi Gaussian Expansion) from its parameters
// (A, sigma, e1, e2, x_c, y_c): value A/(2 pi) exp(-rho^2/(2 sigma^2)).  With
// q = (1-e)/(1+e) and the angle atan2(e2, e1)/2, the elliptical radius
// rho^2 = q x'^2 + y'^2/q of the rotated frame is, in the unrotated offsets,
//   rho^2 = [(1+e^2)(dx^2+dy^2) - 2 e1 (dx^2-dy^2) - 4 e2 dx dy] / (1-e^2)
//         = c1 dx^2 + c2 dy^2 + c3 dx dy,
// which needs no angle and is smooth at e = 0.
struct LightG {
  float A, sig, e1, e2, xc, yc;
  float a2pi;          // A / (2 pi)
  float c1, c2, c3, D; // D = 1/(1-e^2)
  float q1, q2, q3;    // c1..c3 times -log2(e)/(2 sigma^2): the exponent in base 2
};
__device__ __forceinline__ LightG make_light(const float* p) {
  LightG g;
  g.A = p[0]; g.sig = p[1]; g.e1 = p[2]; g.e2 = p[3]; g.xc = p[4]; g.yc = p[5];
  const float ee = g.e1 * g.e1 + g.e2 * g.e2;
  g.D = 1.f / (1.f - ee);
  g.c1 = g.D * (1.f + ee - 2.f * g.e1);
  g.c2 = g.D * (1.f + ee + 2.f * g.e1);
  g.c3 = -4.f * g.D * g.e2;
  g.a2pi = g.A * 0.15915494309189535f;
  const float k2 = -0.72134752044448170f / (g.sig * g.sig);
  g.q1 = k2 * g.c1; g.q2 = k2 * g.c2; g.q3 = k2 * g.c3;
  return g;
}
// Along a row of sub-rays (x = x0 + c h, c < cnt, at fixed y) the base-2
// exponent E(c) = q1 dx^2 + q2 dy^2 + q3 dx dy is quadratic in c, so
// X(c) = 2^E(c) follows from X(c+1) = X(c) R(c), R(c+1) = R(c) Q2 with
// R(0) = 2^(E(1) - E(0)) and Q2 = 2^(2 q1 h^2): two exponentials per row
// instead of one per sub-ray (the relative rounding grows by about one unit
// in the last place per step).  Q2 is per Gaussian and spacing.  Where the
// exponent's change along the row could leave 2^(+-60) (a component far
// narrower than the sub-ray spacing), X would underflow while R overflows;
// such a row takes one exponential per sub-ray instead.
__device__ __forceinline__ float light_q2(const LightG& g, float h) {
  return __builtin_amdgcn_exp2f(2.f * g.q1 * h * h);
}
// Returns false when the row must take the direct exponentials.
__device__ __forceinline__ bool light_row_start(const LightG& g, float x0, float y, float h, int cnt, float& X,
                                                float& R, float& dx0, float& dy) {
  dx0 = x0 - g.xc;
  dy = y - g.yc;
  const float e0 = fmaf(g.q1 * dx0, dx0, fmaf(g.q2 * dy, dy, g.q3 * dx0 * dy));
  const float de = fmaf(g.q1, fmaf(2.f * dx0, h, h * h), g.q3 * dy * h);   // E(1) - E(0)
  X = __builtin_amdgcn_exp2f(e0);
  R = __builtin_amdgcn_exp2f(de);
  return fabsf(de) + 2.f * fabsf(g.q1) * h * h * (float)cnt < 60.f;
}
__device__ __forceinline__ float light_exp_at(const LightG& g, float dx, float dy) {
  return __builtin_amdgcn_exp2f(fmaf(g.q1 * dx, dx, fmaf(g.q2 * dy, dy, g.q3 * dx * dy)));
}
// sum over the row of the Gaussian's value
__device__ __forceinline__ float light_row_sum(const LightG& g, float x0, float y, float h, float q2, int cnt) {
  float X, R, dx0, dy;
  const bool rec = light_row_start(g, x0, y, h, cnt, X, R, dx0, dy);
  float s = 0.f;
  if (rec) {
    for (int c = 0; c < cnt; ++c) {
      s += X;
      X *= R;
      R *= q2;
    }
  } else {
    for (int c = 0; c < cnt; ++c) s += light_exp_at(g, fmaf((float)c, h, dx0), dy);
  }
  return g.a2pi * s;
}
// Moments of X = exp(-rho^2/(2 sigma^2)) over a row, added to
// m = (sum X, sum X dx^2, sum X dy^2, sum X dx dy, sum X dx, sum X dy)
// (dy is constant along the row).
__device__ __forceinline__ void light_row_moments(const LightG& g, float x0, float y, float h, float q2, int cnt,
                                                  float (&m)[6]) {
  float X, R, dx, dy;
  const bool rec = light_row_start(g, x0, y, h, cnt, X, R, dx, dy);
  float sx = 0.f, sxd = 0.f, sxdd = 0.f;
  const float dx0 = dx;
  for (int c = 0; c < cnt; ++c) {
    if (!rec) {
      dx = fmaf((float)c, h, dx0);
      X = light_exp_at(g, dx, dy);
    }
    const float t = X * dx;
    sx += X;
    sxd += t;
    sxdd = fmaf(t, dx, sxdd);
    X *= R;
    R *= q2;
    dx += h;
  }
  m[0] += sx;
  m[1] += sxdd;
  m[2] = fmaf(dy * dy, sx, m[2]);
  m[3] = fmaf(dy, sxd, m[3]);
  m[4] += sxd;
  m[5] = fmaf(dy, sx, m[5]);
}
// d loss / d (A, sigma, e1, e2, x_c, y_c) of one pixel, weight vb = d loss / d
// (sub-ray value), from the moments.  With G = A/(2 pi) X:
//   dG/dA = X/(2 pi), dG/dsigma = G rho^2/sigma^3, and through
//   dG/drho^2 = -G/(2 sigma^2):
//   drho^2/de1 = 2 e1 D rho^2 + D (2 e1 r^2 - 2 (dx^2 - dy^2)),
//   drho^2/de2 = 2 e2 D rho^2 + D (2 e2 r^2 - 4 dx dy),
//   drho^2/dx_c = -(2 c1 dx + c3 dy), drho^2/dy_c = -(2 c2 dy + c3 dx),
// each summed over the sub-rays as a combination of the moments.
__device__ __forceinline__ void light_vjp(const LightG& g, float vb, const float (&m)[6], float (&a)[6]) {
  const float xr2 = g.c1 * m[1] + g.c2 * m[2] + g.c3 * m[3];   // sum X rho^2
  const float xr = m[1] + m[2], xd = m[1] - m[2];                // sum X r^2, sum X (dx^2 - dy^2)
  const float w = vb * g.a2pi, h = -0.5f / (g.sig * g.sig);
  a[0] = vb * 0.15915494309189535f * m[0];
  a[1] = w * xr2 / (g.sig * g.sig * g.sig);
  a[2] = w * h * (2.f * g.e1 * g.D * xr2 + g.D * (2.f * g.e1 * xr - 2.f * xd));
  a[3] = w * h * (2.f * g.e2 * g.D * xr2 + g.D * (2.f * g.e2 * xr - 4.f * m[3]));
  a[4] = -w * h * (2.f * g.c1 * m[4] + g.c3 * m[5]);
  a[5] = -w * h * (2.f * g.c2 * m[5] + g.c3 * m[4]);
}

// ------------------------------------------------------------------ reductions
// Reductions over the 64 lanes of a fully active wave with DPP lane moves
// inside each row of 16 (swap within pairs, within quads, half-row mirror,
// row mirror: every lane of a row then holds the row's result) and the four
// row results read from lanes 0, 16, 32, 48.  No LDS traffic, and a fixed
// order, so the result is the same on every lane and in every run.
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(dpp_move<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  return __hiloint2double(dpp_move<CTRL>(__double2hiint(v)), dpp_move<CTRL>(__double2loint(v)));
}
__device__ __forceinline__ int lane_value(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
template <class T, class OP>
__device__ __forceinline__ T wave_reduce(T v, OP op) {
  v = op(v, dpp_move<0xB1>(v));    // quad_perm [1, 0, 3, 2]
  v = op(v, dpp_move<0x4E>(v));    // quad_perm [2, 3, 0, 1]
  v = op(v, dpp_move<0x141>(v));   // row_half_mirror
  v = op(v, dpp_move<0x140>(v));   // row_mirror
  return op(op(lane_value(v, 0), lane_value(v, 16)), op(lane_value(v, 32), lane_value(v, 48)));
}
__device__ __forceinline__ double wave_sum(double v) {
  return wave_reduce(v, [](double a, double b) { return a + b; });
}
__device__ __forceinline__ float wave_sum(float v) {
  return wave_reduce(v, [](float a, float b) { return a + b; });
}
__device__ __forceinline__ int wave_sum(int v) {
  return wave_reduce(v, [](int a, int b) { return a + b; });
}
__device__ __forceinline__ float wave_min(float v) {
  return wave_reduce(v, [](float a, float b) { return fminf(a, b); });
}
__device__ __forceinline__ float wave_max(float v) {
  return wave_reduce(v, [](float a, float b) { return fmaxf(a, b); });
}
__device__ __forceinline__ int wave_min(int v) {
  return wave_reduce(v, [](int a, int b) { return min(a, b); });
}
__device__ __forceinline__ int wave_max(int v) {
  return wave_reduce(v, [](int a, int b) { return max(a, b); });
}
__device__ __forceinline__ unsigned wave_min(unsigned v) {
  return (unsigned)wave_reduce((int)v, [](int a, int b) { return (int)min((unsigned)a, (unsigned)b); });
}
__device__ __forceinline__ unsigned wave_max(unsigned v) {
  return (unsigned)wave_reduce((int)v, [](int a, int b) { return (int)max((unsigned)a, (unsigned)b); });
}

// Sum of n doubles per thread across the block; result valid in every thread.
// scratch: at least n * (blockDim/64) doubles of LDS.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* scratch) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) scratch[i * nw + wv] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += scratch[i * nw + w];
    v[i] = s;
  }
  __syncthreads();
}

// FP64 column sums of a rows x cols matrix of row stride ld, each in a fixed
// order.  The workgroup reads the matrix row-major (coalesced): thread t takes
// column t % cols and every G-th row from t / cols (G = min(blockDim / cols,
// 16) groups); the G partials of a column are then added in group order.
// `part` is LDS for blockDim doubles.  Called by the whole workgroup.
template <class T, class EMIT>
__device__ __forceinline__ void reduce_columns(const T* a, int rows, int cols, int ld, double* part, EMIT emit) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (cols > nt) {
    for (int c = tid; c < cols; c += nt) {
      double s = 0.0;
      for (int r = 0; r < rows; ++r) s += (double)a[(size_t)r * ld + c];
      emit(c, s);
    }
    __syncthreads();
    return;
  }
  const int G = min(nt / cols, 16);
  const int g = tid / cols, c = tid - g * cols;
  if (g < G) {
    double s = 0.0;
#pragma unroll 8
    for (int r = g; r < rows; r += G) s += (double)a[(size_t)r * ld + c];
    part[tid] = s;
  }
  __syncthreads();
  if (tid < cols) {
    double s = 0.0;
    for (int k = 0; k < G; ++k) s += part[k * cols + tid];
    emit(tid, s);
  }
  __syncthreads();
}

// ------------------------------------------------------------------ FFT
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---- FFT of lines held in LDS: n = N1 * N2 with N1 = min(n, 16), N2 = n / N1,
// each factor a small DFT in registers, so that a line makes two passes
// through LDS.  The natural-order element i = i1 + N1 i2 of a line (i1 < N1)
// is in "split" order stored at N2 i1 + i2.  fft_to_split transforms natural
// input into split-order output; fft_to_natural transforms split-order input
// into natural output (both with W = exp(sign 2 pi i / n)).

// exp(-2 pi i p / 16), p < 8
__device__ __forceinline__ float2 w16(int p) {
  constexpr float C[8] = {1.f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                          0.f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f};
  constexpr float Sn[8] = {0.f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                           -1.f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};
  return make_float2(C[p], Sn[p]);
}

__host__ __device__ constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }
__host__ __device__ constexpr int bitrevc(int i, int l) {
  int r = 0;
  for (int k = 0; k < l; ++k) r |= ((i >> k) & 1) << (l - 1 - k);
  return r;
}

// In-register DFT of N <= 16 points, natural order in and out.
template <int N>
__device__ __forceinline__ void dft_reg(float2* v, float sign) {
  constexpr int L = ilog2c(N);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int j = bitrevc(i, L);
    if (j > i) { const float2 t = v[i]; v[i] = v[j]; v[j] = t; }
  }
#pragma unroll
  for (int s = 1; s <= L; ++s) {
    const int half = 1 << (s - 1);
#pragma unroll
    for (int g = 0; g < N; g += 2 * half) {
#pragma unroll
      for (int q = 0; q < half; ++q) {
        float2 w = w16(q << (4 - s));
        w.y *= -sign;                      // the table holds exp(-i ...): sign +1 conjugates
        const float2 a = v[g + q], b = cmul(v[g + q + half], w);
        v[g + q] = make_float2(a.x + b.x, a.y + b.y);
        v[g + q + half] = make_float2(a.x - b.x, a.y - b.y);
      }
    }
  }
}

// exp(sign 2 pi i e / n) for n <= 256 from the LDS table tw[k] = exp(-2 pi i k / 256)
__device__ __forceinline__ float2 twiddle(const float2* tw, int e, int n, float sign) {
  const int k = (e * (256 / n)) & 255;
  float2 w = tw[k & 127];
  if (k & 128) { w.x = -w.x; w.y = -w.y; }
  w.y *= -sign;
  return w;
}

// A set of nl lines: element j of line l sits at buf[l * ls + j * es].  With
// LFAST the work items run along the lines first (consecutive threads take
// consecutive lines: the right order for columns of a row-major grid),
// otherwise along the elements of one line first.
template <int N1, int N2, bool LFAST>
__device__ __forceinline__ void fft_to_split(float2* buf, const float2* tw, int nl, int ls, int es, float sign) {
  constexpr int n = N1 * N2;
  float2 v[N1 > N2 ? N1 : N2];
  // step 1: for each t < N2, the N1 points t + N2 m
  for (int it = threadIdx.x; it < nl * N2; it += blockDim.x) {
    int l, t;
    if (LFAST) { t = it / nl; l = it - t * nl; } else { l = it / N2; t = it - l * N2; }
    float2* p = buf + l * ls + t * es;
#pragma unroll
    for (int m = 0; m < N1; ++m) v[m] = p[N2 * m * es];
    dft_reg<N1>(v, sign);
#pragma unroll
    for (int k = 1; k < N1; ++k) v[k] = cmul(v[k], twiddle(tw, t * k, n, sign));
#pragma unroll
    for (int k = 0; k < N1; ++k) p[N2 * k * es] = v[k];
  }
  __syncthreads();
  if (N2 > 1) {
    // step 2: for each k1 < N1, the N2 consecutive points N2 k1 + t
    for (int it = threadIdx.x; it < nl * N1; it += blockDim.x) {
      int l, k1;
      if (LFAST) { k1 = it / nl; l = it - k1 * nl; } else { l = it / N1; k1 = it - l * N1; }
      float2* p = buf + l * ls + N2 * k1 * es;
#pragma unroll
      for (int t = 0; t < N2; ++t) v[t] = p[t * es];
      dft_reg<N2>(v, sign);
#pragma unroll
      for (int t = 0; t < N2; ++t) p[t * es] = v[t];
    }
    __syncthreads();
  }
}

template <int N1, int N2, bool LFAST>
__device__ __forceinline__ void fft_to_natural(float2* buf, const float2* tw, int nl, int ls, int es, float sign) {
  constexpr int n = N1 * N2;
  float2 v[N1 > N2 ? N1 : N2];
  if (N2 > 1) {
    // step A: for each i1 < N1, the N2 consecutive points N2 i1 + i2, then W^(i1 k2)
    for (int it = threadIdx.x; it < nl * N1; it += blockDim.x) {
      int l, i1;
      if (LFAST) { i1 = it / nl; l = it - i1 * nl; } else { l = it / N1; i1 = it - l * N1; }
      float2* p = buf + l * ls + N2 * i1 * es;
#pragma unroll
      for (int t = 0; t < N2; ++t) v[t] = p[t * es];
      dft_reg<N2>(v, sign);
#pragma unroll
      for (int k = 1; k < N2; ++k) v[k] = cmul(v[k], twiddle(tw, i1 * k, n, sign));
#pragma unroll
      for (int t = 0; t < N2; ++t) p[t * es] = v[t];
    }
    __syncthreads();
  }
  // step B: for each k2 < N2, the N1 points N2 i1 + k2 (stride N2)
  for (int it = threadIdx.x; it < nl * N2; it += blockDim.x) {
    int l, k2;
    if (LFAST) { k2 = it / nl; l = it - k2 * nl; } else { l = it / N2; k2 = it - l * N2; }
    float2* p = buf + l * ls + k2 * es;
#pragma unroll
    for (int m = 0; m < N1; ++m) v[m] = p[N2 * m * es];
    dft_reg<N1>(v, sign);
#pragma unroll
    for (int k = 0; k < N1; ++k) p[N2 * k * es] = v[k];
  }
  __syncthreads();
}

// position of natural element i of a line in split order
__device__ __forceinline__ int split_pos(int i, int logn) {
  const int l1 = logn < 4 ? logn : 4, n2 = 1 << (logn - l1);
  return n2 * (i & ((1 << l1) - 1)) + (i >> l1);
}

// natural index of the element at split position p of a line
__device__ __forceinline__ int split_nat(int p, int logn) {
  const int l1 = logn < 4 ? logn : 4, l2 = logn - l1;
  return (p >> l2) + ((p & ((1 << l2) - 1)) << l1);
}

// Transform nl lines (element j of line l at buf[l * ls + j * es]) from
// natural to split order (to_split) or from split to natural order.
template <bool LFAST>
__device__ __forceinline__ void fft_lines_dir(float2* buf, const float2* tw, int nl, int logn, int ls, int es,
                                              float sign, bool to_split) {
  switch (logn) {
#define RTU_FFT_CASE(LG, A, B)                                                \
    case LG:                                                                  \
      if (to_split) fft_to_split<A, B, LFAST>(buf, tw, nl, ls, es, sign);     \
      else fft_to_natural<A, B, LFAST>(buf, tw, nl, ls, es, sign);            \
      break;
    RTU_FFT_CASE(3, 8, 1)
    RTU_FFT_CASE(4, 16, 1)
    RTU_FFT_CASE(5, 16, 2)
    RTU_FFT_CASE(6, 16, 4)
    RTU_FFT_CASE(7, 16, 8)
    RTU_FFT_CASE(8, 16, 16)
#undef RTU_FFT_CASE
    default: break;
  }
}

// Rows (cols = false) or columns of an n x n grid held whole in LDS at row
// stride n + 1.  In both directions consecutive threads take consecutive
// lines: rows n + 1 (odd) float2s apart then fall in consecutive LDS bank
// pairs, where the elements of one row, taken along the row, put up to 8
// lanes of a wave on one bank pair (measured at n = 128: a row pass 10 us
// that way, 4.4 us like this, as long as a column pass).
__device__ __forceinline__ void fft_grid_dir(float2* A, const float2* tw, int n, int logn, bool cols, float sign,
                                             bool to_split) {
  if (cols) fft_lines_dir<true>(A, tw, n, logn, 1, n + 1, sign, to_split);
  else fft_lines_dir<true>(A, tw, n, logn, n + 1, 1, sign, to_split);
}

// U-wide batches of independent global loads over [0, tot): v = ld(q), then
// st(q, v) for every q of the thread, so that U loads are in flight at once.
template <int U, class LD, class ST>
__device__ __forceinline__ void batched_copy(int tot, LD ld, ST st) {
  const int nt = blockDim.x;
  for (int base = threadIdx.x; base < tot; base += U * nt) {
    decltype(ld(0)) v[U];
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (base + j * nt < tot) v[j] = ld(base + j * nt);
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (base + j * nt < tot) st(base + j * nt, v[j]);
  }
}

// One pass of a 2-D FFT over an n x n complex array: every row (cols = false)
// or every column (cols = true) is loaded through `ld(row, col)`, transformed
// with sign1, handed to `mid(row, col, value)` (which may rescale it), then
// transformed with sign2 if `twice`, and written through `st(row, col, value)`.
// Lines are processed in chunks that fit the cap float2 slots of the LDS
// buffer, which holds 128 more slots after them for the twiddle table; with
// lend > 0 only the lines [lbeg, lend) are.  The global loads and stores go U
// per thread at a time.
template <int U = 8, class LD, class MID, class ST>
__device__ __forceinline__ void fft_pass(float2* lds, int cap, int n, int logn, bool cols, float sign1, bool twice, float sign2,
                         LD ld, MID mid, ST st, int lbeg = 0, int lend = 0) {
  float2* tw = lds + cap;
  for (int k = threadIdx.x; k < 128; k += blockDim.x) tw[k] = c_tw[k];
  const int ls = n + 1;
  const int nt = blockDim.x;
  const int le = lend > 0 ? lend : n;   // lines [lbeg, le) only
  int chunk = cap / ls;
  if (chunk > n) chunk = n;
  for (int l0 = lbeg; l0 < le; l0 += chunk) {
    const int nl = min(chunk, le - l0);
    const int tot = nl * n;
    // element idx of the chunk: its line l, its index i along the line, and
    // its (row, col) in the array
    auto place = [&](int idx, int& l, int& i, int& row, int& col) {
      if (cols) { l = idx % nl; i = idx / nl; } else { i = idx & (n - 1); l = idx >> logn; }
      row = cols ? i : l0 + l;
      col = cols ? l0 + l : i;
    };
    for (int base = threadIdx.x; base < tot; base += U * nt) {
      float2 v[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        int l, i, row, col;
        if (base + j * nt < tot) {
          place(base + j * nt, l, i, row, col);
          v[j] = ld(row, col);
        }
      }
#pragma unroll
      for (int j = 0; j < U; ++j) {
        int l, i, row, col;
        if (base + j * nt < tot) {
          place(base + j * nt, l, i, row, col);
          lds[l * ls + i] = v[j];
        }
      }
    }
    __syncthreads();
    fft_lines_dir<false>(lds, tw, nl, logn, ls, 1, sign1, true);
    for (int idx = threadIdx.x; idx < tot; idx += nt) {
      int l, i, row, col;
      place(idx, l, i, row, col);
      const int q = l * ls + split_pos(i, logn);
      lds[q] = mid(row, col, lds[q]);
    }
    __syncthreads();
    if (twice) fft_lines_dir<false>(lds, tw, nl, logn, ls, 1, sign2, false);
    for (int base = threadIdx.x; base < tot; base += U * nt) {
      float2 v[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        int l, i, row, col;
        if (base + j * nt < tot) {
          place(base + j * nt, l, i, row, col);
          v[j] = lds[l * ls + (twice ? i : split_pos(i, logn))];
        }
      }
#pragma unroll
      for (int j = 0; j < U; ++j) {
        int l, i, row, col;
        if (base + j * nt < tot) {
          place(base + j * nt, l, i, row, col);
          st(row, col, v[j]);
        }
      }
    }
    __syncthreads();
  }
}

// Signed FFT frequency of index i on an n-grid.
__device__ __forceinline__ float fft_freq(int i, int n) { return (float)(i < (n >> 1) ? i : i - n); }

// log sqrt(P(k)) of the Matern spectrum (eq. 4) and its derivatives in
// (sigma, n, zeta).
struct Matern {
  float lsig, n, zeta, a, c0;  // a = 2n/zeta^2, c0 = log sigma + log(4 pi n)/2 + (n/2) log a
};
__device__ __forceinline__ Matern make_matern(const float* ps) {
  Matern m;
  m.n = ps[1];
  m.zeta = ps[2];
  m.lsig = __logf(ps[0]);
  m.a = 2.f * m.n / (m.zeta * m.zeta);
  m.c0 = m.lsig + 0.5f * __logf(4.f * 3.14159265358979f * m.n) + 0.5f * m.n * __logf(m.a);
  return m;
}
__device__ __forceinline__ float matern_sqrtP(const Matern& m, float k2) {
  return __expf(m.c0 - 0.5f * (m.n + 1.f) * __logf(m.a + k2));
}

}  // namespace rtu
