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
__device__ __forceinline__ float softplus_f(float x) {
  return fmaxf(x, 0.f) + log1pf(__expf(-fabsf(x)));
}
// log(softplus(x)), finite for all x
__device__ __forceinline__ float log_softplus_f(float x) {
  return x < -15.f ? x : __logf(softplus_f(x));
}

// ------------------------------------------------------------------ SIE + shear
// Per-sample constants of the singular isothermal ellipsoid (eq. A1 at slope 2)
// kappa = (theta_E/2) / sqrt(q x'^2 + y'^2/q) and of the external shear.
struct Sie {
  float the, x0, y0, g1, g2;
  float c, s;        // cos, sin of the position angle phi = atan2(e2, e1)/2
  float q, f, P;     // axis ratio, f = sqrt(1-q^2), P = theta_E sqrt(q)
  float e1, e2, e;
};

__device__ __forceinline__ Sie make_sie(const float* L) {
  Sie o;
  o.the = L[0]; o.e1 = L[1]; o.e2 = L[2]; o.x0 = L[3]; o.y0 = L[4]; o.g1 = L[5]; o.g2 = L[6];
  o.e = sqrtf(o.e1 * o.e1 + o.e2 * o.e2);
  o.q = (1.f - o.e) / (1.f + o.e);
  const float phi = 0.5f * atan2f(o.e2, o.e1);
  sincosf(phi, &o.s, &o.c);
  o.f = 2.f * sqrtf(o.e) / (1.f + o.e);   // sqrt(1 - q^2) without cancellation
  o.P = o.the * sqrtf(o.q);
  return o;
}

// atan(f a)/f and its partial derivatives in a and f (series for small f).
__device__ __forceinline__ void atan_over_f(float f, float a, float& v, float& da, float& df) {
  const float fa = f * a;
  const float den = 1.f / (1.f + fa * fa);
  da = den;
  if (f < 1e-3f) {
    v = a * (1.f - fa * fa * (1.f / 3.f));
    df = -(2.f / 3.f) * f * a * a * a;
  } else {
    v = atanf(fa) / f;
    df = (a * den - v) / f;
  }
}
// atanh(f b)/f and its partial derivatives in b and f (|f b| < 1).
__device__ __forceinline__ void atanh_over_f(float f, float b, float& v, float& db, float& df) {
  const float fb = f * b;
  const float den = 1.f / (1.f - fb * fb);
  db = den;
  if (f < 1e-3f) {
    v = b * (1.f + fb * fb * (1.f / 3.f));
    df = (2.f / 3.f) * f * b * b * b;
  } else {
    v = atanhf(fb) / f;
    df = (b * den - v) / f;
  }
}

// Deflection of SIE + shear at (x, y).
__device__ __forceinline__ void sie_shear_alpha(const Sie& L, float x, float y, float& ax, float& ay) {
  const float dx = x - L.x0, dy = y - L.y0;
  const float xp = L.c * dx + L.s * dy;
  const float yp = -L.s * dx + L.c * dy;
  const float psi = sqrtf(L.q * L.q * xp * xp + yp * yp);
  float axp = 0.f, ayp = 0.f;
  if (psi > 1e-20f) {
    const float ip = 1.f / psi;
    float A, dA, fA, B, dB, fB;
    atan_over_f(L.f, xp * ip, A, dA, fA);
    atanh_over_f(L.f, yp * ip, B, dB, fB);
    axp = L.P * A;
    ayp = L.P * B;
  }
  ax = L.c * axp - L.s * ayp + L.g1 * x + L.g2 * y;
  ay = L.s * axp + L.c * ayp + L.g2 * x - L.g1 * y;
}

// Accumulators of the SIE + shear vector-Jacobian product; converted to
// parameter gradients once per tile by sie_grad().
struct SieAcc {
  float P, q, f, phi, x0, y0, g1, g2;
  __device__ __forceinline__ void zero() { P = q = f = phi = x0 = y0 = g1 = g2 = 0.f; }
};

// Given d loss / d alpha at (x, y), accumulate d loss / d (internal SIE
// quantities) and the shear gradient.
__device__ __forceinline__ void sie_shear_vjp(const Sie& L, float x, float y, float abx, float aby,
                                              SieAcc& acc) {
  acc.g1 += abx * x - aby * y;
  acc.g2 += abx * y + aby * x;
  const float dx = x - L.x0, dy = y - L.y0;
  const float xp = L.c * dx + L.s * dy;
  const float yp = -L.s * dx + L.c * dy;
  const float psi = sqrtf(L.q * L.q * xp * xp + yp * yp);
  if (!(psi > 1e-20f)) return;
  const float ip = 1.f / psi;
  const float a = xp * ip, b = yp * ip;
  float A, dA, fA, B, dB, fB;
  atan_over_f(L.f, a, A, dA, fA);
  atanh_over_f(L.f, b, B, dB, fB);
  const float axp = L.P * A, ayp = L.P * B;
  // rotation alpha = R(phi) alpha': d/dphi R(phi) alpha' = (-alpha'_y rot, alpha'_x rot)
  const float rx = L.c * axp - L.s * ayp, ry = L.s * axp + L.c * ayp;
  float phib = abx * (-ry) + aby * rx;
  const float axpb = L.c * abx + L.s * aby;
  const float aypb = -L.s * abx + L.c * aby;
  acc.P += axpb * A + aypb * B;
  const float ab = axpb * L.P * dA;
  const float bb = aypb * L.P * dB;
  acc.f += axpb * L.P * fA + aypb * L.P * fB;
  float xpb = ab * ip, ypb = bb * ip;
  const float psib = -(ab * a + bb * b) * ip;
  acc.q += psib * L.q * xp * xp * ip;
  xpb += psib * L.q * L.q * xp * ip;
  ypb += psib * yp * ip;
  phib += xpb * yp - ypb * xp;
  acc.phi += phib;
  const float dxb = L.c * xpb - L.s * ypb;
  const float dyb = L.s * xpb + L.c * ypb;
  acc.x0 -= dxb;
  acc.y0 -= dyb;
}

// Convert summed accumulators (double) to d loss / d (theta_E, e1, e2, x0, y0, g1, g2).
__device__ __forceinline__ void sie_grad(const Sie& L, const double* a, double* g) {
  // a: P, q, f, phi, x0, y0, g1, g2
  const double sq = sqrt((double)L.q);
  const double e = (double)L.e;
  g[0] = a[0] * sq;
  const double qb = a[1] + a[0] * (double)L.the / (2.0 * sq);
  const double dqde = -2.0 / ((1.0 + e) * (1.0 + e));
  const double dfde = (1.0 - e) / (sqrt(e) * (1.0 + e) * (1.0 + e));
  const double eb = qb * dqde + a[2] * dfde;
  const double e1 = L.e1, e2 = L.e2;
  g[1] = eb * e1 / e - a[3] * e2 / (2.0 * e * e);
  g[2] = eb * e2 / e + a[3] * e1 / (2.0 * e * e);
  g[3] = a[4];
  g[4] = a[5];
  g[5] = a[6];
  g[6] = a[7];
}

// ------------------------------------------------------------------ NFW (App. A.2)
// T(v) = atanh(sqrt v)/sqrt v (v > 0), atan(sqrt(-v))/sqrt(-v) (v < 0), 1 at 0.
__device__ __forceinline__ float nfw_T(float v) {
  if (fabsf(v) < 0.1f) {
    float r = 1.f / 17.f;
    r = fmaf(r, v, 1.f / 15.f); r = fmaf(r, v, 1.f / 13.f); r = fmaf(r, v, 1.f / 11.f);
    r = fmaf(r, v, 1.f / 9.f);  r = fmaf(r, v, 1.f / 7.f);  r = fmaf(r, v, 1.f / 5.f);
    r = fmaf(r, v, 1.f / 3.f);  r = fmaf(r, v, 1.f);
    return r;
  }
  if (v > 0.f) { const float s = sqrtf(v); return atanhf(s) / s; }
  const float s = sqrtf(-v);
  return atanf(s) / s;
}

// Projected-mass function h(X) of the NFW convergence (eq. A3) and h'(X) = X G(X),
// G = (1 - F(X))/(X^2 - 1) = kappa/(2 kappa_s).
__device__ __forceinline__ void nfw_h_dh(float X, float& h, float& dh) {
  if (X < 1e-6f) {
    const float L = __logf(2.f / X);
    h = X * X * (0.5f * L - 0.25f);
    dh = X * (L - 1.f);
    return;
  }
  if (X < 0.5f) {
    const float X2 = X * X;
    const float c = sqrtf(1.f - X2);
    h = __logf(2.f / X) * X2 / ((1.f + c) * c) + log1pf(-X2 / (2.f * (1.f + c))) / c;
    const float F = atanhf(c) / c;
    dh = X * (F - 1.f) / (c * c);
    return;
  }
  const float v = (1.f - X) / (1.f + X);
  h = __logf(0.5f * X) + 2.f * nfw_T(v) / (1.f + X);
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
    G = (nfw_T(vp) - 1.f) / vp;
  }
  dh = X * G;
}

struct Nfw {
  float ks, rs, xs, ys, htau;  // htau = h(tau) (tau > 0)
};

__device__ __forceinline__ Nfw make_nfw(const float* p, float tau) {
  Nfw o;
  o.ks = p[0]; o.rs = p[1]; o.xs = p[2]; o.ys = p[3];
  o.htau = 0.f;
  if (tau > 0.f) { float d; nfw_h_dh(tau, o.htau, d); }
  return o;
}

// alpha = 4 ks rs^2 H(X) d / r^2, d = theta - centre, X = r/rs, H = h(min(X, tau)).
__device__ __forceinline__ void nfw_alpha(const Nfw& N, float tau, float x, float y, float& ax, float& ay) {
  const float dx = x - N.xs, dy = y - N.ys;
  const float r2 = dx * dx + dy * dy;
  if (!(r2 > 1e-30f)) return;
  const float r = sqrtf(r2);
  const float X = r / N.rs;
  float H, dH;
  if (tau > 0.f && X > tau) { H = N.htau; } else { nfw_h_dh(X, H, dH); }
  const float C = 4.f * N.ks * N.rs * N.rs * H / r2;
  ax += C * dx;
  ay += C * dy;
}

// d loss/d(ks, rs, xs, ys) given d loss / d alpha.
__device__ __forceinline__ void nfw_vjp(const Nfw& N, float tau, float x, float y, float abx, float aby,
                                        float& gks, float& grs, float& gxs, float& gys) {
  const float dx = x - N.xs, dy = y - N.ys;
  const float r2 = dx * dx + dy * dy;
  if (!(r2 > 1e-30f)) return;
  const float r = sqrtf(r2);
  const float X = r / N.rs;
  float H, dH;
  if (tau > 0.f && X > tau) { H = N.htau; dH = 0.f; } else { nfw_h_dh(X, H, dH); }
  const float Y = abx * dx + aby * dy;
  const float ir2 = 1.f / r2;
  const float rs = N.rs;
  gks += 4.f * rs * rs * H * Y * ir2;
  grs += Y * 4.f * N.ks * (2.f * rs * H - r * dH) * ir2;
  const float C = 4.f * N.ks * rs * rs * H * ir2;
  // C'(r)/r = 4 ks (rs H'/r^3 - 2 rs^2 H / r^4)
  const float Cpr = 4.f * N.ks * (rs * dH / r - 2.f * rs * rs * H * ir2) * ir2;
  const float dxb = C * abx + Y * Cpr * dx;
  const float dyb = C * aby + Y * Cpr * dy;
  gxs -= dxb;
  gys -= dyb;
}

// ------------------------------------------------------------------ CDF spline
// Number of knots <= z (0..K): the spline interval of z.
__device__ __forceinline__ int knot_count(const float* X, float z) {
  int k = 0;
#pragma unroll
  for (int step = 16; step >= 1; step >>= 1) {
    if (k + step <= K && X[k + step - 1] <= z) k += step;
  }
  return k;
}

// Cubic Hermite spline through (X_k, u_k) with slopes S_k, linear outside.
// Returns g(z); dg = dg/dz.
__device__ __forceinline__ float cdf_eval(const float* X, const float* S, float z, int k, float& dg) {
  if (k == 0) { dg = S[0]; return c_u[0] + S[0] * (z - X[0]); }
  if (k >= K) { dg = S[K - 1]; return c_u[K - 1] + S[K - 1] * (z - X[K - 1]); }
  const int l = k - 1;
  const float Xl = X[l];
  const float h = X[l + 1] - Xl;
  const float ih = 1.f / h;
  const float t = (z - Xl) * ih;
  const float t2 = t * t, t3 = t2 * t;
  const float u0 = c_u[l], u1 = c_u[l + 1];
  const float hs0 = h * S[l], hs1 = h * S[l + 1];
  const float g = u0 + (u1 - u0) * (3.f * t2 - 2.f * t3) + hs0 * (t3 - 2.f * t2 + t) + hs1 * (t3 - t2);
  const float dgdt = (u1 - u0) * (6.f * t - 6.f * t2) + hs0 * (3.f * t2 - 4.f * t + 1.f) + hs1 * (3.f * t2 - 2.f * t);
  dg = dgdt * ih;
  return g;
}

// Partial derivatives of g(z) with respect to the knots and slopes of its
// interval: gXl, gXr (d g/d X_l, X_{l+1}) and gSl, gSr.  For the linear
// continuations only the end knot is involved (returned in the *l slots).
__device__ __forceinline__ void cdf_knot_partials(const float* X, const float* S, float z, int k,
                                                  float& gXl, float& gXr, float& gSl, float& gSr) {
  if (k == 0) { gXl = -S[0]; gSl = z - X[0]; gXr = gSr = 0.f; return; }
  if (k >= K) { gXl = -S[K - 1]; gSl = z - X[K - 1]; gXr = gSr = 0.f; return; }
  const int l = k - 1;
  const float Xl = X[l];
  const float h = X[l + 1] - Xl;
  const float ih = 1.f / h;
  const float t = (z - Xl) * ih;
  const float t2 = t * t, t3 = t2 * t;
  const float u0 = c_u[l], u1 = c_u[l + 1];
  const float h10 = t3 - 2.f * t2 + t, h11 = t3 - t2;
  const float dgdt = (u1 - u0) * (6.f * t - 6.f * t2) + h * S[l] * (3.f * t2 - 4.f * t + 1.f) +
                     h * S[l + 1] * (3.f * t2 - 2.f * t);
  const float gh = h10 * S[l] + h11 * S[l + 1];
  gSl = h * h10;
  gSr = h * h11;
  gXl = dgdt * (t - 1.f) * ih - gh;
  gXr = -dgdt * t * ih + gh;
}

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
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

// ------------------------------------------------------------------ FFT
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place radix-2 transforms of nl lines of length n = 2^logn held in LDS with
// line stride ls, input already in bit-reversed order.  sign = -1 forward
// (e^{-2 pi i k x / n}), +1 inverse; no normalisation.
__device__ __forceinline__ void fft_lines(float2* buf, int nl, int n, int logn, int ls, float sign) {
  const int half_n = n >> 1;
  const int nb = nl * half_n;
  for (int s = 1; s <= logn; ++s) {
    const int half = 1 << (s - 1);
    for (int idx = threadIdx.x; idx < nb; idx += blockDim.x) {
      const int l = idx >> (logn - 1);
      const int k = idx & (half_n - 1);
      const int grp = k >> (s - 1);
      const int pos = k & (half - 1);
      const int i0 = (grp << s) + pos;
      float2 w = c_tw[pos << (8 - s)];
      w.y *= -sign;  // table holds e^{-i}: forward keeps it, inverse conjugates
      float2* p = buf + l * ls;
      const float2 a = p[i0];
      const float2 b = cmul(p[i0 + half], w);
      p[i0] = make_float2(a.x + b.x, a.y + b.y);
      p[i0 + half] = make_float2(a.x - b.x, a.y - b.y);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int bitrev(int i, int logn) {
  return (int)(__brev((unsigned)i) >> (32 - logn));
}

// One pass of a 2-D FFT over an n x n complex array: every row (cols = false)
// or every column (cols = true) is loaded through `ld(row, col)`, transformed
// with sign1, handed to `mid(row, col, value)` (which may rescale it), then
// transformed with sign2 if `twice`, and written through `st(row, col, value)`.
// Lines are processed in chunks that fit the LDS buffer.
template <class LD, class MID, class ST>
__device__ void fft_pass(float2* lds, int n, int logn, bool cols, float sign1, bool twice, float sign2,
                         LD ld, MID mid, ST st) {
  const int ls = n + 1;
  int chunk = FFT_LDS_FLOAT2 / ls;
  if (chunk > n) chunk = n;
  for (int l0 = 0; l0 < n; l0 += chunk) {
    const int nl = min(chunk, n - l0);
    const int tot = nl * n;
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      int l, i;
      if (cols) { l = idx % nl; i = idx / nl; } else { i = idx & (n - 1); l = idx >> logn; }
      const int row = cols ? i : l0 + l, col = cols ? l0 + l : i;
      lds[l * ls + bitrev(i, logn)] = ld(row, col);
    }
    __syncthreads();
    fft_lines(lds, nl, n, logn, ls, sign1);
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      int l, i;
      if (cols) { l = idx % nl; i = idx / nl; } else { i = idx & (n - 1); l = idx >> logn; }
      const int row = cols ? i : l0 + l, col = cols ? l0 + l : i;
      lds[l * ls + i] = mid(row, col, lds[l * ls + i]);
    }
    __syncthreads();
    if (twice) {
      // bit-reverse in place, then transform again
      for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int l = idx >> logn, i = idx & (n - 1);
        const int j = bitrev(i, logn);
        if (j > i) {
          float2* p = lds + l * ls;
          const float2 t = p[i];
          p[i] = p[j];
          p[j] = t;
        }
      }
      __syncthreads();
      fft_lines(lds, nl, n, logn, ls, sign2);
    }
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      int l, i;
      if (cols) { l = idx % nl; i = idx / nl; } else { i = idx & (n - 1); l = idx >> logn; }
      const int row = cols ? i : l0 + l, col = cols ? l0 + l : i;
      st(row, col, lds[l * ls + i]);
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
