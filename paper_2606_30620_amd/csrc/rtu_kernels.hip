// gfx950 kernels of one RTU-grid likelihood evaluation and its adjoint.
//
// Stage order on the caller's stream:
//   k_prep      per sample: arc-masked ray shooting, standardisation, exact
//               quantile selection (histogram + scan + in-bin ranking), the
//               Chebyshev slope fit -> smoothed-CDF knots (App. C i-iv); and,
//               in a third workgroup role, the FFT Gaussian-process source
//               (eqs. 1-4).
//   k_rays_fwd  per 16x16 pixel tile: sub-rays -> lens equation -> RTU
//               transform (eq. 5) -> bilinear source value -> pixel mean.
//   k_psf       PSF correlation through an LDS tile; the forward variant also
//               forms the residual and the chi^2 partial sums (FP64).
//   k_rays_adj  per tile: the same rays again, scattering d loss/d s into an
//               LDS copy of the grid and accumulating d loss/d knots and
//               d loss/d lens parameters.
//   k_post      per sample, two workgroup roles: (0) the loss, the knot
//               adjoint back to the selected masked rays and the lens
//               gradient; (1) the GP adjoint through the FFT.  Each role
//               ORs its status bits into the sample's status word.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>
#include <stdint.h>

#include "rtu_device.h"
#include "rtu_internal.h"

namespace rtu {

__constant__ float c_u[K];
__constant__ double c_ud[K];
__constant__ double c_D[K * K];
__constant__ float2 c_tw[128];

// Masked-pixel count and rank-one PSF flag of the observation: from the
// descriptor, or from the table of an observation prepared on the device.
__device__ __forceinline__ int obs_M(const SysDev& S) { return S.obs_dyn ? S.obs_dyn[0] : S.M; }
__device__ __forceinline__ int obs_rank1(const SysDev& S) { return S.obs_dyn ? S.obs_dyn[1] : S.psf_rank1; }

// ====================================================================== helpers
// Sub-ray (a, b) of pixel (i, j) sits at the pixel centre
// ((j - (N-1)/2) d, (i - (N-1)/2) d) plus (((b + 1/2)/ss - 1/2) d,
// ((a + 1/2)/ss - 1/2) d), i.e. at (x0 + b dxs, y0 + a dxs).
__device__ __forceinline__ void subray_origin(const SysDev& S, int i, int j, float& x0, float& y0, float& dxs) {
  const float inv = 1.f / (float)S.ss;
  x0 = ((float)j + 0.5f * inv - 0.5f * (float)S.n_img) * S.pix;
  y0 = ((float)i + 0.5f * inv - 0.5f * (float)S.n_img) * S.pix;
  dxs = inv * S.pix;
}

__device__ __forceinline__ int n_sub_of(const SysDev& S, int b) {
  if (!S.n_sub || S.n_sub_max == 0) return 0;
  const int v = S.n_sub[b];
  return v < 0 ? 0 : (v > S.n_sub_max ? S.n_sub_max : v);
}

// The main deflector with the external shear: the SIE (slope 2) or, with
// the EPL geometry flag, the elliptical power law (its series tables in LDS).
template <bool EPL> struct Main;
template <> struct Main<false> {
  Sie L;
  __device__ __forceinline__ Main(const float* lensp, const EplTab*) : L(make_sie(lensp)) {}
  __device__ __forceinline__ explicit Main(const Sie& c) : L(c) {}
  __device__ __forceinline__ void alpha(float x, float y, float& ax, float& ay) const {
    sie_shear_alpha(L, x, y, ax, ay);
  }
  // A bound on the spectral norm of d alpha/d theta at distance >= r from the
  // centre: the SIE potential is homogeneous of degree one, so its Hessian
  // has the eigenvalues 0 and 2 kappa = theta_E / rho <= theta_E / (sqrt(q) r)
  // (rho^2 = q x'^2 + y'^2 / q >= q r^2 for q <= 1); the shear adds gamma.
  // Infinite or NaN where no bound holds (r = 0, q <= 0).
  __device__ __forceinline__ float jac_bound(float r) const { return L.jb * rcp(r) + L.gam; }
  __device__ __forceinline__ float cx() const { return L.x0; }
  __device__ __forceinline__ float cy() const { return L.y0; }
};
template <> struct Main<true> {
  Epl L;
  const EplTab* T;
  __device__ __forceinline__ Main(const float* lensp, const EplTab* t) : L(make_epl(lensp)), T(t) {}
  __device__ __forceinline__ void alpha(float x, float y, float& ax, float& ay) const {
    epl_shear_alpha(L, *T, x, y, ax, ay);
  }
  // no bound is used for the power law: its rays are never skipped
  __device__ __forceinline__ float jac_bound(float) const { return INFINITY; }
  __device__ __forceinline__ float cx() const { return L.x0; }
  __device__ __forceinline__ float cy() const { return L.y0; }
};

// The main deflector of sample b in a ray kernel: the SIE from the constants
// its selection workgroup stored, the power law from the lens vector and the
// series tables in LDS.
template <bool EPL>
__device__ __forceinline__ Main<EPL> main_of(const SysDev& S, int b, const float* lensp, const EplTab* t);
template <>
__device__ __forceinline__ Main<false> main_of<false>(const SysDev& S, int b, const float*, const EplTab*) {
  return Main<false>(S.sie[b]);
}
template <>
__device__ __forceinline__ Main<true> main_of<true>(const SysDev&, int, const float* lensp, const EplTab* t) {
  return Main<true>(lensp, t);
}

// beta = theta - alpha(theta) for the main deflector + shear + subhaloes
template <class MAIN>
__device__ __forceinline__ void shoot(const SysDev& S, const MAIN& L, const float* lensp, int nsub,
                                      float x, float y, float& bx, float& by) {
  float ax, ay;
  L.alpha(x, y, ax, ay);
  for (int j = 0; j < nsub; ++j) {
    const Nfw N = make_nfw(lensp + S.lens_base + RTU_N_PER_SUB * j, S.tau);
    nfw_alpha(N, S.tau, x, y, ax, ay);
  }
  bx = x - ax;
  by = y - ay;
}
template <class MAIN>
__device__ __forceinline__ void shoot(const SysDev& S, const MAIN& L, const Nfw* nf, int nsub,
                                      float x, float y, float& bx, float& by) {
  float ax, ay;
  L.alpha(x, y, ax, ay);
  for (int j = 0; j < nsub; ++j) nfw_alpha(nf[j], S.tau, x, y, ax, ay);
  bx = x - ax;
  by = y - ay;
}

// Order-preserving map of a float onto uint32 (-0 taken as +0; NaNs sort
// beyond the infinities, by sign).
__device__ __forceinline__ unsigned ord_key(float v) {
  const unsigned u = __float_as_uint(v + 0.0f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
// Sort key of masked ray m: its value, ties by index.
__device__ __forceinline__ unsigned long long sel_key(float v, int m) {
  return ((unsigned long long)ord_key(v) << 32) | (unsigned)m;
}
// The value of an order key.
__device__ __forceinline__ float ord_value(unsigned k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// ====================================================================== k_prep
// The type-7 quantiles need the masked rays at 2K ranks of their sorted order
// (ties by ray index): floor(h_k) and floor(h_k) + 1 for every node.  Both
// selections below take the distinct ranks in ascending order (L.trank[0,
// ntgt)), made once per observation (target_list) with the map from the
// nodes to it.  First a value-linear histogram over the finite range
// [vmin, vmax] names the bin of every target rank.  When the target bins are
// small, their rays are gathered into LDS and ranked by counting.  Otherwise
// (rays clustered far below the histogram's resolution, many ties,
// non-finite values) a most-significant-digit radix select on the unique keys
//   key(m) = (ord(v_m) - ord_min) << ib | m   (tb = vb + ib bits)
// finds them: every pass histograms the next digit of the rays that share an
// unresolved target's prefix, a target is resolved once its prefix holds one
// ray, and the number of passes is bounded by the key width whatever the
// values are.  The digit width adapts to the number of distinct prefixes so
// that groups x bins fits the LDS histogram.
constexpr int HIST_BINS = 4096;          // first level: value-linear bins
constexpr int SEL_LDS_CAP = 3072;        // rays of the target bins ranked by counting
constexpr int SEL_SEG_MAX = 256;         // largest target bin ranked by counting
constexpr int SEL_BINS = 11264;          // radix: groups << digit bits <= SEL_BINS
constexpr int SEL_MAX_DIGIT = 13;

struct SelLds {
  union {
    struct {
      int hist[HIST_BINS];
      unsigned long long cand[SEL_LDS_CAP];
    } c;
    int rhist[SEL_BINS + 1];
  };
  double red[8 * 16];
  float fred[2 * 16];
  unsigned ured[2 * 16];
  int trank[2 * K];                      // distinct target ranks, ascending: [0, ntgt)
  int tmap[2 * K];                       // rank floor(h_k) + (t & 1) of node t/2 is target tmap[t]
  int ntgt;
  // counting path
  int tbin[2 * K];
  int seg_bin[2 * K], seg_start[2 * K], seg_count[2 * K], seg_fill[2 * K], seg_t0[2 * K];
  int nseg, total, maxcnt;
  // radix path
  unsigned long long gpre[2 * K];        // prefixes of the active groups (ascending)
  unsigned long long tpre[2 * K];        // per target: prefix of its consumed bits
  unsigned long long ulo[2 * K], uhi[2 * K];  // resolved key ranges (ascending, disjoint)
  int tlen[2 * K], tgrp[2 * K], tres[2 * K];
  int ut0[2 * K], ut1[2 * K];
  int ng, nu, consumed, w;
  // result
  float tval[2 * K];
  int tidx[2 * K];
  double q[K];
  float kx[K], ks[K], kd[K];   // the knots, slopes and d p / d u as stored (FP32)
  uint32_t stat;
  EplTab etab;                  // EPL deflector: the sample's series tables
};
// per-wave slots (red, fred, ured: 16 waves) and the weighted sort's per-wave
// digit counts in rhist hold the widest prep workgroup
static_assert(PREP_THREADS_WIDE / 64 <= 16 && 256 * (1 + PREP_THREADS_WIDE / 64) <= SEL_BINS + 1,
              "prep workgroup wider than the selection's LDS");

// Exclusive scan of h[0, n) by the whole workgroup; h[n] = total.
__device__ __forceinline__ void block_exclusive_scan(int* h, int n, int* wsum) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6;
  const int per = (n + nt - 1) / nt;
  const int i0 = min(tid * per, n), i1 = min(i0 + per, n);
  int s = 0;
  for (int i = i0; i < i1; ++i) s += h[i];
  int incl = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  int off = 0;
  for (int q = 0; q < wv; ++q) off += wsum[q];
  int run = off + incl - s;
  for (int i = i0; i < i1; ++i) { const int c = h[i]; h[i] = run; run += c; }
  if (tid == nt - 1) h[n] = off + incl;
  __syncthreads();
}

// Targets t in [0, 2K) with ranks L.trank: rank by counting inside the
// value-linear bins (returns false, having changed nothing but the bin
// histogram, when a target bin is too large for it).
__device__ bool select_by_counting(SelLds& L, const float* zb, int M, float vmin, float vmax) {
  const int tid = threadIdx.x, nt = blockDim.x;
  int* hist = L.c.hist;
  for (int i = tid; i <= HIST_BINS; i += nt) hist[i] = 0;   // hist[HIST_BINS] aliases cand[0]: rewritten below
  __syncthreads();
  const float scale = (vmax > vmin) ? (float)HIST_BINS / (vmax - vmin) : 0.f;
  // monotone in the key order: -NaN, -inf -> 0; +inf, +NaN -> last
  auto bin_of = [&](float v) {
    if (isnan(v)) return signbit(v) ? 0 : HIST_BINS - 1;
    const float t = (v - vmin) * scale;
    if (!(t > 0.f)) return isinf(v) && v > 0.f ? HIST_BINS - 1 : 0;
    return t < (float)HIST_BINS ? (int)t : HIST_BINS - 1;
  };
  batched_copy<8>(M, [&](int m) { return zb[m]; }, [&](int, float v) { atomicAdd(&hist[bin_of(v)], 1); });
  __syncthreads();
  block_exclusive_scan(hist, HIST_BINS, reinterpret_cast<int*>(L.red));
  const int ntgt = L.ntgt;
  if (tid < ntgt) {
    const int r = L.trank[tid];
    int lo = 0, hi = HIST_BINS - 1;   // largest bin with cum <= r
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (hist[mid] <= r) lo = mid; else hi = mid - 1;
    }
    L.tbin[tid] = lo;
  }
  __syncthreads();
  // segments = runs of targets in one bin (the target bins ascend): one wave,
  // lane t for target t; a run starts where the bin changes
  if (tid < 64) {
    const int t = tid;
    const bool valid = t < ntgt;
    const int bb = valid ? L.tbin[t] : -1;
    const int prev = __shfl_up(bb, 1, 64);
    const bool head = valid && (t == 0 || prev != bb);
    const unsigned long long hm = __ballot(head);
    const int cnt = head ? hist[bb + 1] - hist[bb] : 0;
    int incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(incl, o, 64);
      if (t >= o) incl += u;
    }
    const int mx = wave_max(cnt);
    if (head) {
      const int sg = __popcll(hm & ((2ull << t) - 1ull)) - 1;   // heads at lanes <= t, minus one
      L.seg_bin[sg] = bb;
      L.seg_t0[sg] = t;
      L.seg_start[sg] = incl - cnt;
      L.seg_count[sg] = cnt;
      L.seg_fill[sg] = 0;
    }
    if (t == 63) {
      L.nseg = __popcll(hm);
      L.total = incl;
      L.maxcnt = mx;
    }
  }
  __syncthreads();
  const int nseg = L.nseg, total = L.total;
  if (total > SEL_LDS_CAP || L.maxcnt > SEL_SEG_MAX) return false;
  if (tid < ntgt) L.trank[tid] -= hist[L.tbin[tid]];     // rank inside the bin
  __syncthreads();
  // map bin -> segment (reuse the histogram)
  for (int i = tid; i < HIST_BINS; i += nt) hist[i] = -1;
  __syncthreads();
  if (tid < nseg) hist[L.seg_bin[tid]] = tid;
  __syncthreads();
  batched_copy<8>(M, [&](int m) { return zb[m]; }, [&](int m, float v) {
    const int sg = hist[bin_of(v)];
    if (sg >= 0) {
      const int pos = atomicAdd(&L.seg_fill[sg], 1);
      L.c.cand[L.seg_start[sg] + pos] = sel_key(v, m);
    }
  });
  __syncthreads();
  // rank inside each segment by counting, all candidates in parallel; the
  // targets of a segment are a contiguous range of t (ranks are sorted)
  for (int idx = tid; idx < total; idx += nt) {
    int lo = 0, hi = nseg - 1;      // segment holding position idx
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (L.seg_start[mid] <= idx) lo = mid; else hi = mid - 1;
    }
    const int st0 = L.seg_start[lo], cnt = L.seg_count[lo], bb = L.seg_bin[lo];
    const unsigned long long kc = L.c.cand[idx];
    int rk = 0;
    for (int c2 = 0; c2 < cnt; ++c2) rk += L.c.cand[st0 + c2] < kc;
    for (int t = L.seg_t0[lo]; t < ntgt && L.tbin[t] == bb; ++t) {
      if (L.trank[t] == rk) {
        const int m = (int)(kc & 0xffffffffu);
        L.tval[t] = zb[m];
        L.tidx[t] = m;
      }
    }
  }
  __syncthreads();
  return true;
}

// Targets t in [0, 2K) with ranks L.trank: radix select on the unique keys.
__device__ void select_by_radix(SelLds& L, const float* zb, int M, unsigned umin, unsigned umax) {
  const int tid = threadIdx.x, nt = blockDim.x;
  int* hist = L.rhist;
  const unsigned R = umax - umin;
  const int vb = R ? 32 - __clz((int)R) : 0;
  const int ib = M > 1 ? 32 - __clz(M - 1) : 0;
  const int tb = vb + ib;                       // <= 32 + 31 bits
  auto key = [&](int m) {
    return ((unsigned long long)(ord_key(zb[m]) - umin) << ib) | (unsigned)m;
  };
  const int ntgt = L.ntgt;
  if (tid < ntgt) {
    L.tpre[tid] = 0ull;
    L.tlen[tid] = 0;
    L.tres[tid] = tb == 0;                      // a single ray
  }
  __syncthreads();
  for (;;) {
    if (tid == 0) {
      int ng = 0, consumed = tb;
      for (int t = 0; t < ntgt; ++t) {
        if (L.tres[t]) continue;
        if (ng == 0 || L.gpre[ng - 1] != L.tpre[t]) L.gpre[ng++] = L.tpre[t];
        L.tgrp[t] = ng - 1;
        consumed = L.tlen[t];                   // the same for every unresolved target
      }
      int w = 0;
      if (ng) {
        w = SEL_MAX_DIGIT;
        while ((ng << w) > SEL_BINS) --w;
        if (w > tb - consumed) w = tb - consumed;
      }
      L.ng = ng;
      L.consumed = consumed;
      L.w = w;
    }
    __syncthreads();
    const int ng = L.ng, w = L.w, sh = tb - L.consumed - w;
    if (ng == 0) break;
    const int nb = ng << w;
    for (int i = tid; i <= nb; i += nt) hist[i] = 0;
    __syncthreads();
    const unsigned long long dmask = (1ull << w) - 1ull;
    for (int m = tid; m < M; m += nt) {
      const unsigned long long k = key(m);
      const unsigned long long pre = (k >> sh) >> w;
      int lo = 0, hi = ng - 1;                  // the group with this prefix, if any
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.gpre[mid] <= pre) lo = mid; else hi = mid - 1;
      }
      if (L.gpre[lo] == pre) atomicAdd(&hist[(lo << w) + (int)((k >> sh) & dmask)], 1);
    }
    __syncthreads();
    block_exclusive_scan(hist, nb, reinterpret_cast<int*>(L.red));
    if (tid < ntgt && !L.tres[tid]) {
      const int base = L.tgrp[tid] << w;
      const int target = hist[base] + L.trank[tid];
      int lo = 0, hi = (1 << w) - 1;            // largest digit whose start <= target
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (hist[base + mid] <= target) lo = mid; else hi = mid - 1;
      }
      const int cnt = hist[base + lo + 1] - hist[base + lo];
      L.trank[tid] = target - hist[base + lo];
      L.tpre[tid] = (L.tpre[tid] << w) | (unsigned long long)lo;
      L.tlen[tid] += w;
      L.tres[tid] = cnt <= 1 || L.tlen[tid] >= tb;
    }
    __syncthreads();
  }
  // every target's prefix now holds exactly one ray: fetch it
  if (tid == 0) {
    int nu = 0;
    for (int t = 0; t < ntgt; ++t) {
      const int free_bits = tb - L.tlen[t];
      const unsigned long long lo = L.tpre[t] << free_bits;
      if (nu == 0 || L.ulo[nu - 1] != lo) {
        L.ulo[nu] = lo;
        L.uhi[nu] = lo + (1ull << free_bits);
        L.ut0[nu] = t;
        ++nu;
      }
      L.ut1[nu - 1] = t;
    }
    L.nu = nu;
  }
  __syncthreads();
  const int nu = L.nu;
  for (int m = tid; m < M; m += nt) {
    const unsigned long long k = key(m);
    int lo = 0, hi = nu - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (L.ulo[mid] <= k) lo = mid; else hi = mid - 1;
    }
    if (L.ulo[lo] <= k && k < L.uhi[lo]) {
      const float v = zb[m];
      for (int t = L.ut0[lo]; t <= L.ut1[lo]; ++t) { L.tval[t] = v; L.tidx[t] = m; }
    }
  }
  __syncthreads();
}

// The spline tables of one axis for the ray kernels (App. C iv): the Hermite
// pieces g = u_l + du (3t^2 - 2t^3) + h S_l (t^3 - 2t^2 + t) + h S_r (t^3 - t^2)
// as cubics in t, scaled to grid coordinates, with linear continuation by the
// end slopes outside the knots.
// ---- weighted RTU grid (Sec. 6.3): weights count rays, so the order
// statistic at cumulative-weight position r is the ray whose interval
// [C_{i-1}, C_i) of the weights summed in sorted order (ties by index) holds
// r.  The masked rays are sorted by a stable least-significant-digit radix
// sort of their 32-bit order keys (the index order of equal keys is kept) in
// global scratch, then the weights are summed in that order in FP64 chunk by
// chunk and each target position finds its ray.

// Inclusive FP64 sum over the block of v (every thread calls); the block
// total in *total.  wsum: one double per wave of LDS.
__device__ __forceinline__ double block_scan_f64(double v, double* wsum, double* total) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  double incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    const double t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  double off = 0.0, tot = 0.0;
  for (int q = 0; q < nw; ++q) {
    if (q < wv) off += wsum[q];
    tot += wsum[q];
  }
  __syncthreads();
  *total = tot;
  return off + incl;
}

// Stable sort of (order key, ray index) pairs of the M masked rays by key,
// four passes of 8-bit digits between A and Bf; the result is in A.
__device__ void weighted_sort(SelLds& L, uint2* A, uint2* Bf, int M) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
  int* hist = L.rhist;              // [256] digit counts, then the running bases
  int* cnt = L.rhist + 256;         // [nw][256] per-wave digit counts of a chunk (nw <= 16)
  for (int pass = 0; pass < 4; ++pass) {
    const int sh = 8 * pass;
    for (int d = tid; d < 256; d += nt) hist[d] = 0;
    __syncthreads();
    for (int m = tid; m < M; m += nt) atomicAdd(&hist[(A[m].x >> sh) & 255], 1);
    __syncthreads();
    if (tid == 0) {
      int run = 0;
      for (int d = 0; d < 256; ++d) { const int c = hist[d]; hist[d] = run; run += c; }
    }
    __syncthreads();
    for (int c0 = 0; c0 < M; c0 += nt) {
      const int m = c0 + tid;
      const bool valid = m < M;
      const uint2 e = valid ? A[m] : make_uint2(0u, 0u);
      const int d = (int)((e.x >> sh) & 255);
      // lanes of this wave with the same digit: one ballot per digit bit
      unsigned long long same = __ballot(valid);
      for (int bit = 0; bit < 8; ++bit) {
        const unsigned long long on = __ballot(((d >> bit) & 1) != 0);
        same &= ((d >> bit) & 1) ? on : ~on;
      }
      const int local = __popcll(same & ((1ull << lane) - 1ull));
      for (int q = tid; q < nw * 256; q += nt) cnt[q] = 0;
      __syncthreads();
      if (valid && local == 0) cnt[wv * 256 + d] = __popcll(same);
      __syncthreads();
      if (valid) {
        int pos = hist[d] + local;
        for (int q = 0; q < wv; ++q) pos += cnt[q * 256 + d];
        Bf[pos] = e;
      }
      __syncthreads();
      for (int dd = tid; dd < 256; dd += nt) {
        int s = 0;
        for (int q = 0; q < nw; ++q) s += cnt[q * 256 + dd];
        hist[dd] += s;
      }
      __syncthreads();
    }
    uint2* t = A; A = Bf; Bf = t;
  }
}

// The 2K order statistics of the weighted quantiles: target t of node t/2 at
// position wr0[t/2] + (t & 1); results in L.tval / L.tidx with the identity
// map L.tmap.  A target beyond the total weight takes the last ray in sorted
// order.
__device__ __forceinline__ void select_weighted(const SysDev& S, SelLds& L, const float* zb, int M, int b, int axis) {
  const int tid = threadIdx.x, nt = blockDim.x;
  uint2* A = S.wsort + ((size_t)b * 2 + axis) * 2 * M;
  uint2* Bf = A + M;
  for (int m = tid; m < M; m += nt) A[m] = make_uint2(ord_key(zb[m]), (unsigned)m);
  __syncthreads();
  weighted_sort(L, A, Bf, M);
  if (tid < 2 * K) { L.tidx[tid] = -1; L.tmap[tid] = tid; }
  if (tid == 0) L.ntgt = 2 * K;
  double* wsum = reinterpret_cast<double*>(L.c.cand);
  double run = 0.0;
  __syncthreads();
  for (int c0 = 0; c0 < M; c0 += nt) {
    const int m = c0 + tid;
    const uint2 e = m < M ? A[m] : make_uint2(0u, 0u);
    const double w = m < M ? (double)S.ray_w[e.y] : 0.0;
    double tot;
    const double hi = run + block_scan_f64(w, wsum, &tot), lo = hi - w;
    if (m < M && w > 0.0)
      for (int t = 0; t < 2 * K; ++t) {
        const double r = S.wr0[t >> 1] + (double)(t & 1);
        if (lo <= r && r < hi) { L.tidx[t] = (int)e.y; L.tval[t] = zb[e.y]; }
      }
    run += tot;
  }
  __syncthreads();
  if (tid < 2 * K && L.tidx[tid] < 0 && M > 0) {
    const uint2 e = A[M - 1];
    L.tidx[tid] = (int)e.y;
    L.tval[tid] = zb[e.y];
  }
  __syncthreads();
}

// On an affine end piece T = c.x + c.y (z - p.x) p.y: the z at which T
// reaches -2.25 (low end) or n + 1.25 (high end), moved to the piece's own
// side of p.x; -inf / +inf if the slope is not positive.  Every z below (above)
// it has T below (above) that level.
__device__ __forceinline__ float grid_reach(float4 c, float2 p, bool hi, float n) {
  const float sl = c.y * p.y, Tl = hi ? n + 1.25f : -2.25f;
  if (!(sl > 0.f)) return hi ? INFINITY : -INFINITY;
  const float z = p.x + (Tl - c.x) / sl;
  return hi ? fmaxf(z, p.x) : fminf(z, p.x);
}

__device__ __forceinline__ void knot_table(const SysDev& S, int b, int ax, const float* X, const float* Sl,
                                           const float* dp) {
  KnotTab& T = S.ktab[b];
  const int tid = threadIdx.x;
  const float n = (float)S.n_src;
  if (tid < K) {
    T.X[ax][tid] = X[tid];
    T.Sl[ax][tid] = Sl[tid];
    T.dp[ax][tid] = dp[tid];
    T.ih[ax][tid] = tid < K - 1 ? 1.f / (X[tid + 1] - X[tid]) : 0.f;
    if (ax == 0) T.du[tid] = tid < K - 1 ? c_u[tid + 1] - c_u[tid] : 0.f;
  }
  if (tid < 32) T.xs[ax][tid] = tid < K ? X[tid] : INFINITY;
  if (tid <= K) {
    const int k = tid;
    T.kr[ax][k] = make_float2(k == 0 ? -INFINITY : X[k - 1], k == K ? INFINITY : X[k]);
    if (k == 0 || k == K) {
      const int e = k == 0 ? 0 : K - 1;
      T.ct[ax][k] = make_float2(X[e], 1.f);
      T.cq[ax][k] = make_float4(n * c_u[e] - 0.5f, n * Sl[e], 0.f, 0.f);
    } else {
      const int l = k - 1;
      const float h = X[l + 1] - X[l];
      const float du = c_u[l + 1] - c_u[l], hs0 = h * Sl[l], hs1 = h * Sl[l + 1];
      T.ct[ax][k] = make_float2(X[l], 1.f / h);
      T.cq[ax][k] = make_float4(n * c_u[l] - 0.5f, n * hs0, n * (3.f * du - 2.f * hs0 - hs1),
                                n * (hs0 + hs1 - 2.f * du));
    }
  }
  if (tid == 0 || tid == K) {
    const float4 c = T.cq[ax][tid];
    const float2 p = T.ct[ax][tid];
    T.zr[ax][tid == K] = grid_reach(c, p, tid == K, n);
  }
  if (ax == 0 && tid < 2) T.pad[tid] = 0.f;
}

// The uniform grid (Sec. 2.1) in the same tables: one interval [-inf, inf)
// on which the grid coordinate is the affine T = n (z - lo) / L - 1/2, so the
// ray kernels run unchanged and their knot moments of interval 0 are the sums
// of ybar and ybar (z - lo) / L.
__device__ __forceinline__ void knot_table_uniform(const SysDev& S, int b, int ax, float lo, float side) {
  KnotTab& T = S.ktab[b];
  const int tid = threadIdx.x;
  if (tid < K) {
    T.X[ax][tid] = lo; T.Sl[ax][tid] = 1.f / side; T.dp[ax][tid] = side; T.ih[ax][tid] = 0.f;
    if (ax == 0) T.du[tid] = 0.f;
  }
  if (tid < 32) T.xs[ax][tid] = INFINITY;
  if (tid <= K) {
    T.kr[ax][tid] = tid == 0 ? make_float2(-INFINITY, INFINITY) : make_float2(INFINITY, INFINITY);
    T.ct[ax][tid] = make_float2(lo, 1.f / side);
    T.cq[ax][tid] = make_float4(-0.5f, (float)S.n_src, 0.f, 0.f);
    if (tid < 2) T.zr[ax][tid] = grid_reach(T.cq[ax][tid], T.ct[ax][tid], tid == 1, (float)S.n_src);
  }
  if (ax == 0 && tid < 2) T.pad[tid] = 0.f;
}

// The uniform grid's box from the extremes of both axes (keys: value, ties by
// index, per thread), for the axis of this workgroup.  Called by every
// thread.
__device__ __forceinline__ void prep_uniform(const SysDev& S, int b, int axis, SelLds& L, unsigned long long kx0,
                             unsigned long long kx1, unsigned long long ky0, unsigned long long ky1, int M,
                             uint32_t st) {
  const int tid = threadIdx.x;
  if (tid < 2) { L.ulo[tid] = ~0ull; L.uhi[tid] = 0ull; }
  __syncthreads();
  atomicMin(&L.ulo[0], kx0); atomicMax(&L.uhi[0], kx1);
  atomicMin(&L.ulo[1], ky0); atomicMax(&L.uhi[1], ky1);
  __syncthreads();
  const double x0 = M > 0 ? (double)ord_value((unsigned)(L.ulo[0] >> 32)) : 0.0;
  const double x1 = M > 0 ? (double)ord_value((unsigned)(L.uhi[0] >> 32)) : 0.0;
  const double y0 = M > 0 ? (double)ord_value((unsigned)(L.ulo[1] >> 32)) : 0.0;
  const double y1 = M > 0 ? (double)ord_value((unsigned)(L.uhi[1] >> 32)) : 0.0;
  const unsigned long long klo = axis == 0 ? L.ulo[0] : L.ulo[1], khi = axis == 0 ? L.uhi[0] : L.uhi[1];
  const double rx = x1 - x0, ry = y1 - y0;
  double side = rx >= ry ? rx : ry, lox, loy;
  if (M < 2 || !(side > 0.0)) {
    st |= RTU_ST_MASK_SMALL;
    side = 1.0;
    lox = x0;
    loy = y0;
  } else {
    lox = 0.5 * (x0 + x1) - 0.5 * side;
    loy = 0.5 * (y0 + y1) - 0.5 * side;
  }
  knot_table_uniform(S, b, axis, (float)(axis == 0 ? lox : loy), (float)side);
  float* kn = S.knots + ((size_t)b * 2 + axis) * 2 * K;
  float* kd = S.kdbg + ((size_t)b * 2 + axis) * 2 * K;
  int* sel = S.sel + ((size_t)b * 2 + axis) * 2 * K;
  if (tid < 2 * K) {
    kn[tid] = 0.f;
    kd[tid] = 0.f;
    sel[tid] = M > 0 && tid < 2 ? (int)(unsigned)(tid == 0 ? klo : khi) : 0;
  }
  if (tid < K) S.dp[((size_t)b * 2 + axis) * K + tid] = -1.f;
  if (tid == 0) {
    if (axis == 0) {
      double* sd = S.stdv + (size_t)b * 4;
      sd[0] = lox; sd[1] = loy; sd[2] = side; sd[3] = rx >= ry ? 0.0 : 1.0;
    }
    S.st[b * ST_WORDS + axis] = st;
  }
}

// The masked rays at the observed pixel centres (not supersampled): their
// coordinate on this workgroup's axis into zb, the (weighted) moments of
// both axes, the value and key ranges, and the uniform grid's extremes.
struct MaskedRays {
  double sx = 0.0, sy = 0.0, sxx = 0.0, syy = 0.0;
  float vmin = INFINITY, vmax = -INFINITY;      // over the finite values
  unsigned umin = 0xffffffffu, umax = 0u;       // key range over all values
  unsigned long long kx0 = ~0ull, kx1 = 0ull, ky0 = ~0ull, ky1 = 0ull;
};
template <class MAIN>
__device__ __forceinline__ void masked_rays(const SysDev& S, const MAIN& ML, const float* lensp, int nsub, int axis,
                                            int M, float* zb, MaskedRays& R) {
  const int tid = threadIdx.x, nt = blockDim.x;
  // the pixel centre of the iteration after next is loaded ahead
  const float* xy = reinterpret_cast<const float*>(S.mask_xy);
  float p1x = 0.f, p1y = 0.f, p2x = 0.f, p2y = 0.f;
  if (tid < M) { p1x = xy[2 * tid]; p1y = xy[2 * tid + 1]; }
  if (tid + nt < M) { p2x = xy[2 * (tid + nt)]; p2y = xy[2 * (tid + nt) + 1]; }
  for (int m = tid; m < M; m += nt) {
    const float x = p1x, y = p1y;
    p1x = p2x; p1y = p2y;
    if (m + 2 * nt < M) { p2x = xy[2 * (m + 2 * nt)]; p2y = xy[2 * (m + 2 * nt) + 1]; }
    float bx, by;
    shoot(S, ML, lensp, nsub, x, y, bx, by);
    if (S.ray_w) {   // weighted grid: weighted moments
      const double wm = (double)S.ray_w[m];
      R.sx += wm * bx; R.sy += wm * by; R.sxx += wm * bx * bx; R.syy += wm * by * by;
    } else {
      R.sx += bx; R.sy += by; R.sxx += (double)bx * bx; R.syy += (double)by * by;
    }
    const float v = (axis == 0 ? bx : by) + 0.0f;
    zb[m] = v;
    if (isfinite(v)) {
      R.vmin = fminf(R.vmin, v);
      R.vmax = fmaxf(R.vmax, v);
    }
    const unsigned u = ord_key(v);
    R.umin = min(R.umin, u);
    R.umax = max(R.umax, u);
    if (S.uniform) {
      const unsigned long long kx = sel_key(bx, m), ky = sel_key(by, m);
      R.kx0 = min(R.kx0, kx); R.kx1 = max(R.kx1, kx);
      R.ky0 = min(R.ky0, ky); R.ky1 = max(R.ky1, ky);
    }
  }
}

// Chunk c of the masked rays of sample b (a launch before the selection, for
// large masks): the rays m in [c MR_CHUNK, (c + 1) MR_CHUNK), both axes'
// values into zbuf and the chunk's moments and ranges into mrp, with the
// arithmetic of masked_rays.
struct MRayLds {
  EplTab etab;
  double red[4 * (MR_THREADS / 64)];
  float fred[4 * (MR_THREADS / 64)];
  unsigned ured[4 * (MR_THREADS / 64)];
  unsigned long long kred[4];   // uniform grid: x min, x max, y min, y max keys
};
template <class MAIN>
__device__ __forceinline__ void mrays_chunk(const SysDev& S, const MAIN& ML, const float* lensp, int nsub, int b,
                                            int c, MRayLds& L) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
  const int M = S.M, m0 = c * MR_CHUNK, m1 = min(M, m0 + MR_CHUNK);
  float* zx = S.zbuf + (size_t)b * 2 * M;
  float* zy = zx + M;
  const float* xy = reinterpret_cast<const float*>(S.mask_xy);
  double sx = 0.0, sy = 0.0, sxx = 0.0, syy = 0.0;
  float v0x = INFINITY, v1x = -INFINITY, v0y = INFINITY, v1y = -INFINITY;
  unsigned u0x = 0xffffffffu, u1x = 0u, u0y = 0xffffffffu, u1y = 0u;
  unsigned long long kx0 = ~0ull, kx1 = 0ull, ky0 = ~0ull, ky1 = 0ull;
  for (int m = m0 + tid; m < m1; m += nt) {
    const float x = xy[2 * m], y = xy[2 * m + 1];
    float bx, by;
    shoot(S, ML, lensp, nsub, x, y, bx, by);
    if (S.ray_w) {
      const double wm = (double)S.ray_w[m];
      sx += wm * bx; sy += wm * by; sxx += wm * bx * bx; syy += wm * by * by;
    } else {
      sx += bx; sy += by; sxx += (double)bx * bx; syy += (double)by * by;
    }
    const float vx = bx + 0.0f, vy = by + 0.0f;
    zx[m] = vx;
    zy[m] = vy;
    if (isfinite(vx)) { v0x = fminf(v0x, vx); v1x = fmaxf(v1x, vx); }
    if (isfinite(vy)) { v0y = fminf(v0y, vy); v1y = fmaxf(v1y, vy); }
    const unsigned ux = ord_key(vx), uy = ord_key(vy);
    u0x = min(u0x, ux); u1x = max(u1x, ux);
    u0y = min(u0y, uy); u1y = max(u1y, uy);
    if (S.uniform) {
      const unsigned long long kx = sel_key(bx, m), ky = sel_key(by, m);
      kx0 = min(kx0, kx); kx1 = max(kx1, kx);
      ky0 = min(ky0, ky); ky1 = max(ky1, ky);
    }
  }
  if (S.uniform) {
    atomicMin(&L.kred[0], kx0); atomicMax(&L.kred[1], kx1);
    atomicMin(&L.kred[2], ky0); atomicMax(&L.kred[3], ky1);
  }
  double v4[4] = {sx, sy, sxx, syy};
  block_sum<4>(v4, L.red);
  const float f[4] = {wave_min(v0x), wave_min(v0y), wave_max(v1x), wave_max(v1y)};
  const unsigned u[4] = {wave_min(u0x), wave_min(u0y), wave_max(u1x), wave_max(u1y)};
  if (lane == 0)
    for (int q = 0; q < 4; ++q) { L.fred[4 * wv + q] = f[q]; L.ured[4 * wv + q] = u[q]; }
  __syncthreads();
  if (tid == 0) {
    MRayPart P;
    for (int q = 0; q < 4; ++q) P.s[q] = v4[q];
    P.vmin[0] = P.vmin[1] = INFINITY; P.vmax[0] = P.vmax[1] = -INFINITY;
    P.umin[0] = P.umin[1] = 0xffffffffu; P.umax[0] = P.umax[1] = 0u;
    for (int q = 0; q < 4; ++q) P.k[q] = L.kred[q];
    for (int w = 0; w < nw; ++w) {
      const float* fw = L.fred + 4 * w;
      const unsigned* uw = L.ured + 4 * w;
      for (int a = 0; a < 2; ++a) {
        P.vmin[a] = fminf(P.vmin[a], fw[a]); P.vmax[a] = fmaxf(P.vmax[a], fw[2 + a]);
        P.umin[a] = min(P.umin[a], uw[a]); P.umax[a] = max(P.umax[a], uw[2 + a]);
      }
    }
    S.mrp[(size_t)b * S.mr_nchunk + c] = P;
  }
}
__device__ __forceinline__ void mrays_body(const SysDev& S, int b, int c, MRayLds& L) {
  const float* lensp = S.lens + (size_t)b * S.n_lens;
  const int nsub = n_sub_of(S, b);
  if (threadIdx.x == 0) {
    if (S.epl) epl_table(make_epl(lensp), L.etab);
    L.kred[0] = L.kred[2] = ~0ull;
    L.kred[1] = L.kred[3] = 0ull;
  }
  __syncthreads();
  if (S.epl) {
    mrays_chunk(S, Main<true>(lensp, &L.etab), lensp, nsub, b, c, L);
  } else {
    mrays_chunk(S, Main<false>(lensp, nullptr), lensp, nsub, b, c, L);
  }
}
__global__ void __launch_bounds__(MR_THREADS) k_mrays(SysDev S) {
  __shared__ MRayLds L;
  mrays_body(S, blockIdx.y, blockIdx.x, L);
}

__device__ __forceinline__ void prep_select(const SysDev& S, int b, int axis, unsigned char* smem) {
  SelLds& L = *reinterpret_cast<SelLds*>(smem);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
  const int M = obs_M(S);
  const float* lensp = S.lens + (size_t)b * S.n_lens;
  const int nsub = n_sub_of(S, b);
  if (S.epl && tid == 0) epl_table(make_epl(lensp), L.etab);
  if (!S.epl && axis == 0 && tid == 64) S.sie[b] = make_sie(lensp);   // for the ray kernels
  float* zb = S.zbuf + ((size_t)b * 2 + axis) * M;
  uint32_t st = 0;
  if (M < (S.uniform ? 2 : K + 1)) st |= RTU_ST_MASK_SMALL;
  if (tid == 0) L.stat = 0;
  if (tid < 2 * K) { L.tval[tid] = 0.f; L.tidx[tid] = 0; }
  // the selection's targets (read after the reductions' barriers)
  if (tid < 2 * K) { L.trank[tid] = S.tsel[tid]; L.tmap[tid] = S.tsel[2 * K + tid]; }
  if (tid == 0) L.ntgt = S.tsel[4 * K];
  __syncthreads();   // the EPL tables

  MaskedRays R;
  if (S.mr_nchunk) {
    // shot by the masked-ray launch: this thread's chunks, in chunk order
    for (int c = tid; c < S.mr_nchunk; c += nt) {
      const MRayPart& P = S.mrp[(size_t)b * S.mr_nchunk + c];
      R.sx += P.s[0]; R.sy += P.s[1]; R.sxx += P.s[2]; R.syy += P.s[3];
      R.vmin = fminf(R.vmin, P.vmin[axis]); R.vmax = fmaxf(R.vmax, P.vmax[axis]);
      R.umin = min(R.umin, P.umin[axis]); R.umax = max(R.umax, P.umax[axis]);
      R.kx0 = min(R.kx0, P.k[0]); R.kx1 = max(R.kx1, P.k[1]);
      R.ky0 = min(R.ky0, P.k[2]); R.ky1 = max(R.ky1, P.k[3]);
    }
  } else if (S.epl) {
    masked_rays(S, Main<true>(lensp, &L.etab), lensp, nsub, axis, M, zb, R);
  } else {
    masked_rays(S, Main<false>(lensp, nullptr), lensp, nsub, axis, M, zb, R);
  }
  double sx = R.sx, sy = R.sy, sxx = R.sxx, syy = R.syy;
  float vmin = R.vmin, vmax = R.vmax;
  unsigned umin = R.umin, umax = R.umax;
  {
    double v4[4] = {sx, sy, sxx, syy};
    block_sum<4>(v4, L.red);
    sx = v4[0]; sy = v4[1]; sxx = v4[2]; syy = v4[3];
    float a = wave_min(vmin), c = wave_max(vmax);
    umin = wave_min(umin);
    umax = wave_max(umax);
    if (lane == 0) { L.fred[wv] = a; L.fred[16 + wv] = c; L.ured[wv] = umin; L.ured[16 + wv] = umax; }
    __syncthreads();
    vmin = INFINITY; vmax = -INFINITY;
    for (int w = 0; w < nw; ++w) {
      vmin = fminf(vmin, L.fred[w]);
      vmax = fmaxf(vmax, L.fred[16 + w]);
      umin = min(umin, L.ured[w]);
      umax = max(umax, L.ured[16 + w]);
    }
    __syncthreads();
  }
  if (S.uniform) {
    prep_uniform(S, b, axis, L, R.kx0, R.kx1, R.ky0, R.ky1, M, st);
    return;
  }
  const double Md = S.ray_w ? (S.wsum > 0.0 ? S.wsum : 1.0) : (double)(M > 0 ? M : 1);
  const double mux = sx / Md, muy = sy / Md;
  const double sdx = sqrt(fmax(sxx / Md - mux * mux, 0.0));
  const double sdy = sqrt(fmax(syy / Md - muy * muy, 0.0));
  const double sc = fmin(sdx, sdy);
  const double mu = axis == 0 ? mux : muy;

  if (M > 0 && S.ray_w) {
    select_weighted(S, L, zb, M, b, axis);
  } else if (M > 0) {
    // the targets (target_list, made with the observation) are in LDS
    if (S.sel_radix || !select_by_counting(L, zb, M, vmin, vmax)) select_by_radix(L, zb, M, umin, umax);
  }
  __syncthreads();

  // ---- Chebyshev slopes and knots (FP64), App. C steps iii-iv
  float* kn = S.knots + ((size_t)b * 2 + axis) * 2 * K;
  float* kd = S.kdbg + ((size_t)b * 2 + axis) * 2 * K;
  float* dpo = S.dp + ((size_t)b * 2 + axis) * K;
  int* sel = S.sel + ((size_t)b * 2 + axis) * 2 * K;
  const bool degenerate = !(sc > 0.0) || M < 2;
  if (tid < K) {
    double qb;
    const int t0 = M > 0 ? L.tmap[2 * tid] : 0, t1 = M > 0 ? L.tmap[2 * tid + 1] : 0;
    if (M > 0) {
      const double t = S.ray_w ? S.wt[tid] : S.rank_t[tid];
      qb = (1.0 - t) * (double)L.tval[t0] + t * (double)L.tval[t1];
    } else {
      qb = 0.0;
    }
    L.q[tid] = degenerate ? (double)c_u[tid] : (qb - mu) / sc;  // standardised quantile
    sel[2 * tid] = M > 0 ? L.tidx[t0] : 0;
    sel[2 * tid + 1] = M > 0 ? L.tidx[t1] : 0;
  }
  __syncthreads();
  if (tid < K) {
    const double* q = L.q;
    double dpz = 0.0;
    for (int l = 0; l < K; ++l) dpz += c_D[tid * K + l] * q[l];
    const double eps = 1e-6 * (q[K - 1] - q[0]);
    bool bad = !(dpz > eps);
    if (tid < K - 1 && !(q[tid + 1] > q[tid])) bad = true;
    const bool clamp = !(dpz > eps);
    if (bad || degenerate) atomicOr(&L.stat, RTU_ST_NONMONOTONE);
    const double dpc = clamp ? (eps > 0 ? eps : 1.0) : dpz;
    const double scd = degenerate ? 1.0 : sc;
    const double mud = degenerate ? 0.0 : mu;
    kd[tid] = (float)q[tid];
    kd[K + tid] = (float)(1.0 / dpc);
    L.kx[tid] = kn[tid] = (float)(mud + scd * q[tid]);
    L.ks[tid] = kn[K + tid] = (float)(1.0 / (scd * dpc));
    L.kd[tid] = dpo[tid] = clamp ? -1.f : (float)(scd * dpc);
  }
  __syncthreads();
  knot_table(S, b, axis, L.kx, L.ks, L.kd);
  if (tid == 0) {
    if (axis == 0) {
      double* sd = S.stdv + (size_t)b * 4;
      sd[0] = mux; sd[1] = muy; sd[2] = sc; sd[3] = (double)M;
    }
    S.st[b * ST_WORDS + axis] = st | L.stat;
  }
}

// The field value f at point q of sample b and the source s = (s0
// softplus(f/s0))^alpha, s0 = 0.01 (eqs. 1-4), also into the zero-bordered copy.
__device__ __forceinline__ void gp_source(const SysDev& S, int b, int q, float f, float alpha) {
  const int n = S.n_src, logn = S.log2_src;
  const size_t n2 = (size_t)n * n;
  S.fld[(size_t)b * n2 + q] = f;
  const float x = f * 100.f;   // f / s0
  const float s = __expf(alpha * (-4.605170186f + log_softplus_f(x)));
  S.src[(size_t)b * n2 + q] = s;
  S.srcp[(size_t)b * (n + 2) * (n + 2) + ((q >> logn) + 1) * (n + 2) + (q & (n - 1)) + 1] = s;
}

// GP source (eqs. 1-4): F = DFT(w); f = Re IDFT(sqrt(P) F)/n^2; s = (s0 softplus(f/s0))^alpha
__device__ __forceinline__ void prep_gp(const SysDev& S, int b, unsigned char* smem, int cap) {
  float2* lds = reinterpret_cast<float2*>(smem);
  const int n = S.n_src, logn = S.log2_src, n2 = n * n;
  const float* w = S.latent + (size_t)b * n2;
  float2* F = S.F + (size_t)b * n2;
  float* sp = S.srcp + (size_t)b * (n + 2) * (n + 2);
  const float* ps = S.ps + (size_t)b * 4;
  // zero border of the padded copy of s
  for (int q = threadIdx.x; q < 4 * (n + 1); q += blockDim.x) {
    const int side = q / (n + 1), o = q - side * (n + 1);
    const int r = side == 0 ? 0 : (side == 1 ? n + 1 : (side == 2 ? o + 1 : o));
    const int c = side == 0 ? o : (side == 1 ? o + 1 : (side == 2 ? 0 : n + 1));
    sp[r * (n + 2) + c] = 0.f;
  }
  // zero the adjoint accumulator of this sample for the ray adjoint
  if (S.want_grad) {
    double* sb = S.sbar + (size_t)b * n2;
    for (int i = threadIdx.x; i < n2; i += blockDim.x) sb[i] = 0.0;
  }
  // parameter domain
  if (threadIdx.x == 0) {
    const float* L = S.lens + (size_t)b * S.n_lens;
    uint32_t st = 0;
    if (!(L[0] > 0.f) || !(L[1] * L[1] + L[2] * L[2] < 1.f)) st |= RTU_ST_DOMAIN;
    if (S.epl && !(L[7] > 1.f && L[7] < 3.f)) st |= RTU_ST_DOMAIN;
    const int ns = n_sub_of(S, b);
    for (int j = 0; j < ns; ++j)
      if (!(L[S.lens_base + RTU_N_PER_SUB * j + 1] > 0.f)) st |= RTU_ST_DOMAIN;
    for (int g = 0; g < S.n_gauss; ++g) {
      const float* lg = L + S.light_off + RTU_N_PER_GAUSS * g;
      if (!(lg[1] > 0.f) || !(lg[2] * lg[2] + lg[3] * lg[3] < 1.f)) st |= RTU_ST_DOMAIN;
    }
    if (!(ps[0] > 0.f) || !(ps[1] > 0.f) || !(ps[2] > 0.f)) st |= RTU_ST_DOMAIN;
    S.st[b * ST_WORDS + 2] = st;
    S.status[b] = 0u;             // the post roles OR their words into it
  }
  if (gp_split(n)) return;   // the transform: three line-pass launches (gp_pass)
  const Matern mt = make_matern(ps);
  const float alpha = ps[3];
  const float inv_n2 = 1.f / (float)n2;
  auto positivity = [&](int q, float f) { gp_source(S, b, q, f, alpha); };
  {
    // grids below the split size: the whole grid in LDS at row stride n + 1:
    // rows, then columns, to split order; F kept in that layout; times
    // sqrt(P); columns, then rows, back
    float2* tw = lds + cap;
    for (int k = threadIdx.x; k < 128; k += blockDim.x) tw[k] = c_tw[k];
    const int ls = n + 1;
    // four consecutive points of a row per item (n >= 8), all of a thread's
    // loads in flight at once for n <= 128
    batched_copy<8>(n2 >> 2, [&](int q4) { return reinterpret_cast<const float4*>(w)[q4]; },
                    [&](int q4, float4 v) {
                      float2* row = lds + ((4 * q4) >> logn) * ls + ((4 * q4) & (n - 1));
                      row[0] = make_float2(v.x, 0.f); row[1] = make_float2(v.y, 0.f);
                      row[2] = make_float2(v.z, 0.f); row[3] = make_float2(v.w, 0.f);
                    });
    __syncthreads();
    fft_grid_dir(lds, tw, n, logn, false, -1.f, true);
    fft_grid_dir(lds, tw, n, logn, true, -1.f, true);
    for (int q = threadIdx.x; q < n2; q += blockDim.x) {
      const int rs = q >> logn, cs = q & (n - 1);
      const float2 v = lds[rs * ls + cs];
      F[q] = v;
      const float kx = fft_freq(split_nat(cs, logn), n), ky = fft_freq(split_nat(rs, logn), n);
      const float sq = matern_sqrtP(mt, kx * kx + ky * ky);
      lds[rs * ls + cs] = make_float2(v.x * sq, v.y * sq);
    }
    __syncthreads();
    fft_grid_dir(lds, tw, n, logn, true, 1.f, false);
    fft_grid_dir(lds, tw, n, logn, false, 1.f, false);
    for (int q = threadIdx.x; q < n2; q += blockDim.x)
      positivity(q, lds[(q >> logn) * ls + (q & (n - 1))].x * inv_n2);
  }
}

// Dynamic LDS of the prep kernels: the larger of the selection layout and the
// FFT buffer (fft_cap float2 line slots, then the twiddle table).
__global__ void __launch_bounds__(PREP_THREADS_WIDE) k_prep(SysDev S, int fft_cap) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x, role = blockIdx.y;
  if (role < 2) prep_select(S, b, role, smem);
  else prep_gp(S, b, smem, fft_cap);
}

// ====================================================================== ray tiles
// A workgroup takes a 16 x 16 tile of pixels, one pixel per thread.  Wave w
// takes the 8 x 8 quarter (w / 2, w % 2) of the tile, lane l its row l / 8 and
// column l % 8.
__device__ __forceinline__ void ray_pixel(int ti, int tj, int& i, int& j) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  i = ti * RAY_TILE + 8 * (w >> 1) + (l >> 3);
  j = tj * RAY_TILE + 8 * (w & 1) + (l & 7);
}
// Source grid staged in LDS with a one-cell zero border:
// padded index (i + 1) * (n + 2) + (j + 1) for i, j in [-1, n].
struct RayLdsHead : KnotTab {
  double km[2][K + 1][4];   // per axis and knot interval: the tile's knot moments, then
                            // in place their knot adjoint (km_knots)
  Nfw nfw[RTU_MAX_SUB];
  EplTab epl;               // EPL deflector: series tables of the sample
};

// The sample's spline tables into LDS (one 16-byte load per thread), the
// knot-adjoint accumulators zeroed, the subhalo constants.
__device__ __forceinline__ void load_knots(const SysDev& S, int b, RayLdsHead& H) {
  {
    const int ns = n_sub_of(S, b);
    const float* lensp = S.lens + (size_t)b * S.n_lens;
    if ((int)threadIdx.x < ns) H.nfw[threadIdx.x] = make_nfw(lensp + S.lens_base + RTU_N_PER_SUB * threadIdx.x, S.tau);
    if (S.epl && threadIdx.x == 64) epl_table(make_epl(lensp), H.epl);
  }
  const float4* src = reinterpret_cast<const float4*>(S.ktab + b);
  float4* dst = reinterpret_cast<float4*>(static_cast<KnotTab*>(&H));
  for (int i = threadIdx.x; i < (int)(sizeof(KnotTab) / 16); i += blockDim.x) dst[i] = src[i];
  for (int i = threadIdx.x; i < 2 * (K + 1) * 4; i += blockDim.x) (&H.km[0][0][0])[i] = 0.0;
}

// Interval of z on axis ax (the number of knots <= z), trying the previous
// sub-ray's interval k first, then its neighbour on the side z left by; the
// wave runs the (branch-free) binary search only if one of its lanes is still
// outside.
__device__ __forceinline__ int knot_find(const RayLdsHead& H, int ax, float z, int k) {
  const float2 r = H.kr[ax][k];
  const bool ok = r.x <= z && z < r.y;
  if (__any(!ok)) {
    const int k1 = z < r.x ? max(k - 1, 0) : (z >= r.y ? min(k + 1, K) : k);
    const float2 r1 = H.kr[ax][k1];
    const bool ok1 = r1.x <= z && z < r1.y;
    if (__any(!ok1)) {
      int s = 0;
#pragma unroll
      for (int step = 16; step >= 1; step >>= 1) s = H.xs[ax][s + step - 1] <= z ? s + step : s;
      k = ok1 ? k1 : min(s, K);
    } else {
      k = k1;
    }
  }
  return k;
}

// Grid coordinate T = n g(z) - 1/2 of the CDF spline on interval k, its local
// coordinate t and, with D, dT/dz.
template <bool D>
__device__ __forceinline__ float cdf_grid(const RayLdsHead& H, int ax, int k, float z, float& t, float& dT) {
  const float4 c = H.cq[ax][k];
  const float2 p = H.ct[ax][k];
  t = (z - p.x) * p.y;
  if (D) dT = fmaf(fmaf(3.f * c.w, t, 2.f * c.z), t, c.y) * p.y;
  return fmaf(fmaf(fmaf(c.w, t, c.z), t, c.y), t, c.x);
}

// bilinear weights at grid coordinates (tx, ty) = n y - 1/2 (nodes at
// (j + 1/2)/n); returns false if all four corners lie outside the zero-padded
// grid.
struct Bil {
  int i0, j0;
  float fx, fy;
};
__device__ __forceinline__ bool bil_setup(float tx, float ty, int n, Bil& o) {
  if (!(tx >= -1.f && tx < (float)n && ty >= -1.f && ty < (float)n)) return false;
  const float fj = floorf(tx), fi = floorf(ty);
  o.j0 = (int)fj; o.i0 = (int)fi;
  o.fx = tx - fj; o.fy = ty - fi;
  return true;
}

// The four corner values from a zero-bordered copy of the grid (in LDS or in
// global memory), padded index (i + 1) (n + 2) + (j + 1).
__device__ __forceinline__ void bil_corners(const float* g, int n, const Bil& B, float& s00, float& s01,
                                            float& s10, float& s11) {
  const int np = n + 2;
  const int p = (B.i0 + 1) * np + (B.j0 + 1);
  s00 = g[p]; s01 = g[p + 1]; s10 = g[p + np]; s11 = g[p + np + 1];
}

// The corner values are read from the zero-bordered grid in global memory
// (through L1/L2): staging the grid in LDS per tile cost more than it saved.
// Each wave also records a range of source cells that holds every cell its
// sub-rays fell in (tbox): per pixel the range of its sub-rays' grid
// coordinates, kept if it reaches within one cell of the zero-bordered grid
// and clipped to it.  An empty range tells the adjoint that the wave's
// sub-rays contribute nothing to the gradient but lens light (the one-cell
// margin covers the adjoint's own rounding of the same rays); the range sizes
// the adjoint's LDS window when the source grid does not fit in LDS.
// Whether every sub-ray of pixel (i, j) lands off the source grid.  Along a
// segment that keeps a distance >= r from every deflector's centre, beta =
// theta - alpha(theta) moves by at most (1 + ||d alpha/d theta||) times the
// segment's length.  The main deflector bounds its part (jac_bound); a
// subhalo, axisymmetric with a convergence that does not increase outwards,
// has the Hessian eigenvalues kappa_bar and 2 kappa - kappa_bar, both at most
// kappa_bar(r) = |alpha(r)| / r in size, and kappa_bar does not increase with r.
// The sub-rays lie in the pixel square, so all of them land within R = (half
// diagonal) (1 + bound) of the pixel centre's beta.  If that disc lies beyond
// T = -2.25 or T = n + 1.25 on one axis (KnotTab::zr: a quarter cell past the
// per-pixel range test below), every sub-ray falls outside the zero-bordered grid and
// fails that test: the sub-ray loop would add nothing and record nothing.
// (1.001 R + 1e-5 and the quarter cell absorb the FP32 rounding of both
// sides.)  Any NaN leaves the pixel to the loop.
template <bool EPL>
__device__ __forceinline__ bool pixel_off_grid(const SysDev& S, const RayLdsHead& H, const Main<EPL>& L, int nsub,
                                               int i, int j) {
  if (EPL) return false;
  const float h = 0.5f * S.pix;
  const float xc = ((float)j + 0.5f - 0.5f * (float)S.n_img) * S.pix;
  const float yc = ((float)i + 0.5f - 0.5f * (float)S.n_img) * S.pix;
  auto dist = [&](float cx, float cy) {
    const float dx = fmaxf(fabsf(xc - cx) - h, 0.f), dy = fmaxf(fabsf(yc - cy) - h, 0.f);
    return fsqrt(dx * dx + dy * dy);
  };
  const float r = dist(L.cx(), L.cy());
  float bound = r > 0.f ? 1.f + L.jac_bound(r) : INFINITY;
  for (int q = 0; q < nsub; ++q) {
    const Nfw& N = H.nfw[q];
    // kappa_bar taken a little inside, at 0.99 rs (the FP32 offset from the
    // centre then stays below rs), times 1.01
    const float rs = dist(N.xs, N.ys);
    if (!(rs > 1e-3f)) return false;
    float ax = 0.f, ay = 0.f;
    nfw_alpha(N, S.tau, N.xs + 0.99f * rs, N.ys, ax, ay);
    bound += 1.0203f * fabsf(ax) * rcp(rs);
  }
  const float R = fmaf(0.70710678f * S.pix * bound, 1.001f, 1e-5f);
  float bx, by;
  shoot(S, L, H.nfw, nsub, xc, yc, bx, by);
  return bx + R < H.zr[0][0] || bx - R > H.zr[0][1] || by + R < H.zr[1][0] || by - R > H.zr[1][1];
}

template <bool EPL>
__device__ void rays_fwd_body(const SysDev& S, int b, int tile, unsigned char* smem) {
  RayLdsHead& H = *reinterpret_cast<RayLdsHead*>(smem);
  const int ti = tile / S.ray_tx, tj = tile - ti * S.ray_tx;
  int i, j;
  ray_pixel(ti, tj, i, j);
  load_knots(S, b, H);
  __syncthreads();
  const bool in = i < S.n_img && j < S.n_img;
  int bi0 = 1 << 30, bj0 = 1 << 30, bi1 = -(1 << 30), bj1 = -(1 << 30);
  if (in) {
    const float* lensp = S.lens + (size_t)b * S.n_lens;
    const int nsub = n_sub_of(S, b);
    const Main<EPL> L = main_of<EPL>(S, b, lensp, &H.epl);
    const int n = S.n_src;
    const float* gsrc = S.srcp + (size_t)b * (n + 2) * (n + 2);
    float acc = 0.f;
    int kx = 0, ky = 0;
    float x0, y0, dxs;
    subray_origin(S, i, j, x0, y0, dxs);
    float tx0 = INFINITY, tx1 = -INFINITY, ty0 = INFINITY, ty1 = -INFINITY;   // NaN ignored
    const int nss = pixel_off_grid<EPL>(S, H, L, nsub, i, j) ? 0 : S.ss;
    for (int a = 0; a < nss; ++a) {
      const float y = fmaf((float)a, dxs, y0);
      for (int cc = 0; cc < S.ss; ++cc) {
        const int c = (a & 1) ? S.ss - 1 - cc : cc;   // serpentine: neighbouring sub-rays in turn
        const float x = fmaf((float)c, dxs, x0);
        float bx, by;
        shoot(S, L, H.nfw, nsub, x, y, bx, by);
        kx = knot_find(H, 0, bx, kx);
        ky = knot_find(H, 1, by, ky);
        float tx, ty, dTx, dTy;
        const float Tx = cdf_grid<false>(H, 0, kx, bx, tx, dTx);
        const float Ty = cdf_grid<false>(H, 1, ky, by, ty, dTy);
        tx0 = fminf(tx0, Tx); tx1 = fmaxf(tx1, Tx);
        ty0 = fminf(ty0, Ty); ty1 = fmaxf(ty1, Ty);
        Bil B;
        if (bil_setup(Tx, Ty, n, B)) {
          float s00, s01, s10, s11;
          bil_corners(gsrc, n, B, s00, s01, s10, s11);
          acc += (1.f - B.fy) * ((1.f - B.fx) * s00 + B.fx * s01) + B.fy * ((1.f - B.fx) * s10 + B.fx * s11);
        }
      }
    }
    const float hi = (float)(n + 1), top = (float)(n - 1);
    if (tx1 >= -2.f && tx0 < hi && ty1 >= -2.f && ty0 < hi) {
      bi0 = (int)fminf(fmaxf(floorf(ty0), -1.f), top); bi1 = (int)fminf(fmaxf(floorf(ty1), -1.f), top);
      bj0 = (int)fminf(fmaxf(floorf(tx0), -1.f), top); bj1 = (int)fminf(fmaxf(floorf(tx1), -1.f), top);
    }
    // lens light at the same sub-ray positions (not lensed)
    for (int g = 0; g < S.n_gauss; ++g) {
      const LightG G = make_light(lensp + S.light_off + RTU_N_PER_GAUSS * g);
      const float q2 = light_q2(G, dxs);
      for (int a = 0; a < S.ss; ++a) acc += light_row_sum(G, x0, fmaf((float)a, dxs, y0), dxs, q2, S.ss);
    }
    S.u[(size_t)b * S.n_img * S.n_img + i * S.n_img + j] = acc * S.inv_ss2;
  }
  // every lane of the wave is here
  bi0 = wave_min(bi0);
  bj0 = wave_min(bj0);
  bi1 = wave_max(bi1);
  bj1 = wave_max(bj1);
  if ((threadIdx.x & 63) == 0)
    S.tbox[((size_t)b * S.ray_tiles + tile) * (RAY_THREADS / 64) + (threadIdx.x >> 6)] = make_int4(bi0, bj0, bi1, bj1);
}

template <bool EPL>
__global__ void __launch_bounds__(RAY_THREADS) k_rays_fwd(SysDev S) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x / S.ray_tiles;
  rays_fwd_body<EPL>(S, b, blockIdx.x - b * S.ray_tiles, smem);
}

// SUB: the variant for systems with subhaloes, which keeps each subhalo's r,
// h and h' in registers from the deflection to its vector-Jacobian product.
template <bool LDSGRID, bool EPL, bool SUB = false>
__device__ void rays_adj_body(const SysDev& S, int b, int tile, unsigned char* smem) {
  RayLdsHead& H = *reinterpret_cast<RayLdsHead*>(smem);
  const int n = S.n_src, np = n + 2;
  // the source grid is read from its zero-bordered copy through L1/L2 here;
  // only d loss / d s lives in LDS, accumulated in FP64 so that its value does
  // not depend on the order of the atomic additions (to FP32 rounding)
  // padded grid (LDSGRID), else the tile's window of the grid
  double* gb = reinterpret_cast<double*>(smem + sizeof(RayLdsHead));
  float* subacc = reinterpret_cast<float*>(gb + (LDSGRID ? np * np : S.adj_wcap));   // [4 n_sub_max][256]
  const int ti = tile / S.ray_tx, tj = tile - ti * S.ray_tx;
  int i, j;
  ray_pixel(ti, tj, i, j);
  // the cells the forward pass's sub-rays fell in, per wave: a wave whose
  // range is empty has no sub-ray on (or near) the grid, whose d loss / d
  // beta is zero; a tile of such waves without lens light only clears its
  // partials
  const int4* tb = S.tbox + ((size_t)b * S.ray_tiles + tile) * (RAY_THREADS / 64);
  int r0 = 1 << 30, c0 = 1 << 30, r1 = -(1 << 30), c1 = -(1 << 30);
  for (int w = 0; w < RAY_THREADS / 64; ++w) {
    const int4 v = tb[w];
    r0 = min(r0, v.x); c0 = min(c0, v.y); r1 = max(r1, v.z); c1 = max(c1, v.w);
  }
  if (r0 > r1 && S.n_gauss == 0) {
    double* lp = S.lpart + ((size_t)b * S.ray_tiles + tile) * (RAY_THREADS / 64) * (S.n_lens + 2);
    for (int q = threadIdx.x; q < (RAY_THREADS / 64) * (S.n_lens + 2); q += blockDim.x) lp[q] = 0.0;
    double* kbo = S.kbar + ((size_t)b * S.ray_tiles + tile) * 4 * K;
    for (int q = threadIdx.x; q < 4 * K; q += blockDim.x) kbo[q] = 0.0;
    return;
  }
  const int4 wbox = tb[threadIdx.x >> 6];
  const bool wave_on = wbox.x <= wbox.z;
  load_knots(S, b, H);
  // grid in LDS: the points of the cells in the forward's ranges widened by
  // one cell on each side (the same rays, rounded in other code here, stay
  // within), padded rows pr0 .. pr1 and columns pc0 .. pc1
  const int pr0 = max(r0 - 1, -1) + 1, pr1 = min(r1 + 1, n - 1) + 2;
  const int pc0 = max(c0 - 1, -1) + 1, pc1 = min(c1 + 1, n - 1) + 2;
  const int pw = pc1 - pc0 + 1, ph = pr1 - pr0 + 1;
  if (LDSGRID && r0 <= r1)
    for (int q = threadIdx.x; q < ph * pw; q += blockDim.x) {
      const int rr = q / pw;
      gb[(pr0 + rr) * np + pc0 + q - rr * pw] = 0.0;
    }
  // grid in global memory: d loss / d s of the grid points (rows wr0 .. wr0 +
  // wrs, columns wc0 .. wc0 + wcs) around the cells the forward's sub-rays of
  // this tile fell in is summed in LDS, and added to the sample's grid once;
  // a point outside that window, or every point of a tile whose window
  // exceeds the capacity, is added to global memory at once
  int wr0 = 0, wc0 = 0, wrs = 0, wcs = 0;
  if (!LDSGRID) {
    r0 = max(r0, 0); c0 = max(c0, 0); r1 = min(r1 + 1, n - 1); c1 = min(c1 + 1, n - 1);   // cell corners
    if (r1 >= r0 && c1 >= c0 && (long)(r1 - r0 + 1) * (long)(c1 - c0 + 1) <= (long)S.adj_wcap) {
      wr0 = r0; wc0 = c0; wrs = r1 - r0 + 1; wcs = c1 - c0 + 1;
    }
    for (int q = threadIdx.x; q < wrs * wcs; q += blockDim.x) gb[q] = 0.0;
  }
  for (int q = threadIdx.x; q < 4 * S.n_sub_max * RAY_THREADS; q += blockDim.x) subacc[q] = 0.f;
  __syncthreads();
  const float* lensp = S.lens + (size_t)b * S.n_lens;
  const int nsub = n_sub_of(S, b);
  const Main<EPL> M = main_of<EPL>(S, b, lensp, &H.epl);
  const float* gsrc = S.srcp + (size_t)b * np * np;
  double* gsb = S.sbar + (size_t)b * n * n;
  SieAcc acc;                         // SIE: raw accumulators (sie_grad_one)
  acc.zero();
  float eacc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};   // EPL: the parameter gradients
  int ongrid = 0;   // sub-rays of this pixel on the grid
  if (wave_on && i < S.n_img && j < S.n_img) {
    const float vb = S.ubar[(size_t)b * S.n_img * S.n_img + i * S.n_img + j] * S.inv_ss2;
    KnotMom cx{-1, 0.f, 0.f, 0.f, 0.f}, cy{-1, 0.f, 0.f, 0.f, 0.f};
    int kx = 0, ky = 0;
    // d loss / d s of the cell the last sub-rays fell in, kept in registers
    // and added to the grid when the cell changes (sub-rays of one pixel
    // mostly share a cell)
    int ci = -1000, cj = -1000;
    float c00 = 0.f, c01 = 0.f, c10 = 0.f, c11 = 0.f;
    auto flush_cell = [&]() {
      if (ci < -1) return;
      if (LDSGRID && (unsigned)(ci + 1 - pr0) < (unsigned)(ph - 1) && (unsigned)(cj + 1 - pc0) < (unsigned)(pw - 1)) {
        const int p = (ci + 1) * np + (cj + 1);
        atomicAdd(&gb[p], (double)c00);
        atomicAdd(&gb[p + 1], (double)c01);
        atomicAdd(&gb[p + np], (double)c10);
        atomicAdd(&gb[p + np + 1], (double)c11);
      } else {
        // global-memory grid, or (never, by the window's construction) a
        // cell outside the LDS window
        auto add = [&](int ii, int jj, float v) {
          if (ii >= 0 && ii < n && jj >= 0 && jj < n) {
            const int wi = ii - wr0, wj = jj - wc0;
            if (!LDSGRID && (unsigned)wi < (unsigned)wrs && (unsigned)wj < (unsigned)wcs)
              atomicAdd(&gb[wi * wcs + wj], (double)v);
            else
              atomicAdd(&gsb[ii * n + jj], (double)v);
          }
        };
        add(ci, cj, c00); add(ci, cj + 1, c01); add(ci + 1, cj, c10); add(ci + 1, cj + 1, c11);
      }
      c00 = c01 = c10 = c11 = 0.f;
    };
    float x0, y0, dxs;
    subray_origin(S, i, j, x0, y0, dxs);
    for (int a = 0; a < S.ss; ++a) {
      const float y = fmaf((float)a, dxs, y0);
      for (int cc = 0; cc < S.ss; ++cc) {
        const int c = (a & 1) ? S.ss - 1 - cc : cc;   // serpentine order
        const float x = fmaf((float)c, dxs, x0);
        SieRay E;
        float ax, ay;
        if constexpr (EPL) M.alpha(x, y, ax, ay);
        else sie_shear_alpha<true>(M.L, x, y, ax, ay, E);
        float kr[SUB ? RTU_MAX_SUB : 1], kh[SUB ? RTU_MAX_SUB : 1], kdh[SUB ? RTU_MAX_SUB : 1];
        if constexpr (SUB) {
#pragma unroll
          for (int q = 0; q < RTU_MAX_SUB; ++q)
            if (q < nsub) nfw_alpha_keep(H.nfw[q], S.tau, x, y, ax, ay, kr[q], kh[q], kdh[q]);
        } else {
          for (int q = 0; q < nsub; ++q) nfw_alpha(H.nfw[q], S.tau, x, y, ax, ay);
        }
        const float bx = x - ax, by = y - ay;
        kx = knot_find(H, 0, bx, kx);
        ky = knot_find(H, 1, by, ky);
        float tx, ty, dTx, dTy;
        const float Tx = cdf_grid<true>(H, 0, kx, bx, tx, dTx);
        const float Ty = cdf_grid<true>(H, 1, ky, by, ty, dTy);
        Bil B;
        if (!bil_setup(Tx, Ty, n, B)) continue;
        ++ongrid;
        float s00, s01, s10, s11;
        bil_corners(gsrc, n, B, s00, s01, s10, s11);
        // d loss / d s at the four corners
        if (B.i0 != ci || B.j0 != cj) { flush_cell(); ci = B.i0; cj = B.j0; }
        const float w01 = B.fx * (1.f - B.fy), w11 = B.fx * B.fy;
        c00 += vb * ((1.f - B.fy) - w01);
        c01 += vb * w01;
        c10 += vb * (B.fy - w11);
        c11 += vb * w11;
        // d loss / d T (grid coordinates) and d loss / d g = n d loss / d T
        const float Tbx = vb * ((1.f - B.fy) * (s01 - s00) + B.fy * (s11 - s10));
        const float Tby = vb * ((1.f - B.fx) * (s10 - s00) + B.fx * (s11 - s01));
        const float ybx = Tbx * (float)n, yby = Tby * (float)n;
        // knots and slopes of the CDF splines (moments per interval)
        if (kx != cx.k) { km_flush(cx, &H.km[0][0][0]); cx.k = kx; }
        km_add(cx, ybx, tx);
        if (ky != cy.k) { km_flush(cy, &H.km[1][0][0]); cy.k = ky; }
        km_add(cy, yby, ty);
        // d loss / d beta -> d loss / d alpha = -d loss / d beta
        const float abx = -Tbx * dTx, aby = -Tby * dTy;
        if constexpr (EPL) epl_shear_vjp(M.L, *M.T, x, y, abx, aby, eacc);
        else sie_shear_vjp(M.L, E, x, y, abx, aby, acc);
        if constexpr (SUB) {
#pragma unroll
          for (int q = 0; q < RTU_MAX_SUB; ++q)
            if (q < nsub) {
              float* sa = subacc + (4 * q) * RAY_THREADS + threadIdx.x;
              float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f;
              nfw_vjp_kept(H.nfw[q], x, y, abx, aby, kr[q], kh[q], kdh[q], g0, g1, g2, g3);
              sa[0] += g0; sa[RAY_THREADS] += g1; sa[2 * RAY_THREADS] += g2; sa[3 * RAY_THREADS] += g3;
            }
        } else {
          for (int q = 0; q < nsub; ++q) {
            float* sa = subacc + (4 * q) * RAY_THREADS + threadIdx.x;
            float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f;
            nfw_vjp(H.nfw[q], S.tau, x, y, abx, aby, g0, g1, g2, g3);
            sa[0] += g0; sa[RAY_THREADS] += g1; sa[2 * RAY_THREADS] += g2; sa[3 * RAY_THREADS] += g3;
          }
        }
      }
    }
    flush_cell();
    km_flush(cx, &H.km[0][0][0]);
    km_flush(cy, &H.km[1][0][0]);
  }
  // ---- lens-gradient partials of this tile, one row per wave: the raw SIE
  //      and shear accumulators (P, q, f, phi, x0, y0, g1, g2), then the
  //      subhalo sums; the chain to the lens parameters is linear in them and
  //      is applied once per sample, after the sums
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* lp = S.lpart + (((size_t)b * S.ray_tiles + tile) * (RAY_THREADS / 64) + wave) * (S.n_lens + 2);
    float v[8] = {acc.P, acc.q, acc.f, acc.phi, acc.x0, acc.y0, acc.g1, acc.g2};
    if constexpr (EPL)
      for (int k = 0; k < 8; ++k) v[k] = eacc[k];
    float r[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = wave_sum(v[k]);
    const int on = wave_sum(ongrid);
    if (lane == 0) {
      for (int k = 0; k < 8; ++k) lp[k] = (double)r[k];
      if (EPL) lp[8] = 0.0;           // rows: the 8 model terms, then lens index + 1
      lp[S.n_lens + 1] = (double)on;
    }
    for (int q = 0; q < 4 * S.n_sub_max; ++q) {
      const float sq = wave_sum(subacc[q * RAY_THREADS + threadIdx.x]);
      if (lane == 0) lp[S.lens_base + 1 + q] = (double)sq;
    }
    // lens-light gradients: every lane of the wave takes part in the sums,
    // a pixel outside the image with weight zero
    if (S.n_gauss) {
      const bool in = i < S.n_img && j < S.n_img;
      const float vbl = in ? S.ubar[(size_t)b * S.n_img * S.n_img + i * S.n_img + j] * S.inv_ss2 : 0.f;
      float x0, y0, dxs;
      subray_origin(S, i, j, x0, y0, dxs);
      for (int g = 0; g < S.n_gauss; ++g) {
        const LightG G = make_light(lensp + S.light_off + RTU_N_PER_GAUSS * g);
        float m[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, a[6];
        const float q2 = light_q2(G, dxs);
        for (int ai = 0; ai < S.ss; ++ai) light_row_moments(G, x0, fmaf((float)ai, dxs, y0), dxs, q2, S.ss, m);
        light_vjp(G, vbl, m, a);
#pragma unroll
        for (int k = 0; k < RTU_N_PER_GAUSS; ++k) {
          const float r = wave_sum(a[k]);
          if (lane == 0) lp[S.light_off + 1 + RTU_N_PER_GAUSS * g + k] = (double)r;
        }
      }
    }
  }
  // every wave's knot-moment and window atomics are done before they are read
  __syncthreads();
  // knot partials of this tile: the adjoint of each interval, then per knot
  // the intervals it bounds (dX (x), dS (x), dX (y), dS (y))
  if (!S.uniform && threadIdx.x < 2 * (K + 1)) {
    const int ax = threadIdx.x / (K + 1), k = threadIdx.x - ax * (K + 1);
    double v[4];
    km_knots(k, H.km[ax][k], H.X[ax], H.Sl[ax], H.ih[ax], H.du, v);
    for (int c = 0; c < 4; ++c) H.km[ax][k][c] = v[c];
  }
  __syncthreads();
  double* kbo = S.kbar + ((size_t)b * S.ray_tiles + tile) * 4 * K;
  if (S.uniform) {   // the raw moments m0, m1 of the one interval, per axis
    for (int q = threadIdx.x; q < 4 * K; q += blockDim.x) {
      const int ax = q / (2 * K), rem = q - ax * 2 * K;
      kbo[q] = rem < 2 ? H.km[ax][0][rem] : 0.0;
    }
  } else for (int q = threadIdx.x; q < 4 * K; q += blockDim.x) {
    const int ax = q / (2 * K), rem = q - ax * 2 * K, o = rem >= K ? 2 : 0, j = rem - (o ? K : 0);
    const double (*kv)[4] = H.km[ax];
    double v = 0.0;
    if (j <= K - 2) v += kv[j + 1][o];        // left knot of Hermite interval j + 1
    if (j >= 1) v += kv[j][o + 1];            // right knot of Hermite interval j
    if (j == 0) v += kv[0][o];                // linear continuation below X_0
    if (j == K - 1) v += kv[K][o];            // linear continuation above X_{K-1}
    kbo[q] = v;
  }
  // d loss / d s: add the window of the LDS grid (its points inside the
  // grid) to the sample's grid
  if (LDSGRID && r0 <= r1) {
    const int i0 = max(pr0 - 1, 0), j0 = max(pc0 - 1, 0), i1 = min(pr1 - 1, n - 1), j1 = min(pc1 - 1, n - 1);
    const int wj = j1 - j0 + 1, wi = i1 - i0 + 1;
    if (wj > 0 && wi > 0) {
      for (int q = threadIdx.x; q < wi * wj; q += blockDim.x) {
        const int ii = i0 + q / wj, jj = j0 + q % wj;
        const double v = gb[(ii + 1) * np + jj + 1];
        if (v != 0.0) atomicAdd(&gsb[ii * n + jj], v);
      }
    }
  } else {
    for (int q = threadIdx.x; q < wrs * wcs; q += blockDim.x) {
      const double v = gb[q];
      if (v != 0.0) {
        const int r = q / wcs;
        atomicAdd(&gsb[(wr0 + r) * n + wc0 + (q - r * wcs)], v);
      }
    }
  }
}

template <bool LDSGRID, bool EPL>
__global__ void __launch_bounds__(RAY_THREADS) k_rays_adj(SysDev S) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x / S.ray_tiles;
  rays_adj_body<LDSGRID, EPL>(S, b, blockIdx.x - b * S.ray_tiles, smem);
}
template <bool LDSGRID, bool EPL>
__global__ void __launch_bounds__(RAY_THREADS) k_rays_adj_sub(SysDev S) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x / S.ray_tiles;
  rays_adj_body<LDSGRID, EPL, true>(S, b, blockIdx.x - b * S.ray_tiles, smem);
}

// ====================================================================== PSF
// out[i, j] = sum_{a,b} W[a, b] in[i + a - h, j + b - h] (zero outside), h = (KP-1)/2.
// Forward: in = u, W = flipped PSF (a convolution), also r = (m - d)/sigma^2 and
// chi^2 partials.  Adjoint: in = r, W = PSF (the transpose of the convolution).
// The correlation runs on the matrix cores.  For a block of 16 x 16 outputs
// (x: column, y: row) and PSF row a it is a product with a banded Toeplitz
// matrix of the weights:
//   out[y][x] += sum_k T_a[x][k] in[y + a][x0 + k],  T_a[x][k] = W[a][k - x] (0 outside [0, KP)),
// k < 4 psf_nk(KP) (at least 15 + KP), as psf_nk(KP) steps of
// v_mfma_f32_16x16x4_f32 per PSF row (FP32 products and sums).

// residual, model and chi^2 partials of 4 output pixels (forward), or the
// adjoint image (adjoint), then the tile's FP64 chi^2 sums
__device__ __forceinline__ void psf_epilogue(const SysDev& S, int b, int tile, int adjoint, int ty0, int tx0,
                                             int ly, int lx, const float (&acc)[4], double* red) {
  const int N = S.n_img;
  const int gi = ty0 + ly, gj0 = tx0 + lx;
  double c2 = 0.0, c2m = 0.0;
  if ((N & 3) == 0 && gi < N && gj0 + 3 < N) {
    // four whole columns, 16-byte aligned (N and gj0 multiples of 4): vector
    // loads and stores, the same arithmetic in the same order
    const int pi = gi * N + gj0;
    const size_t p = (size_t)b * N * N + pi;
    if (adjoint) {
      *reinterpret_cast<float4*>(S.ubar + p) = make_float4(acc[0], acc[1], acc[2], acc[3]);
    } else {
      const float4 d = *reinterpret_cast<const float4*>(S.image + pi);
      const float4 iv = *reinterpret_cast<const float4*>(S.inv_var + pi);
      const uchar4 mk = *reinterpret_cast<const uchar4*>(S.mask + pi);
      const float dd[4] = {d.x, d.y, d.z, d.w}, ivv[4] = {iv.x, iv.y, iv.z, iv.w};
      const bool mm[4] = {mk.x != 0, mk.y != 0, mk.z != 0, mk.w != 0};
      float rr[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float res = acc[q] - dd[q];
        rr[q] = res * ivv[q];
        const double e = (double)res * (double)res * (double)ivv[q];
        c2 += e;
        if (mm[q]) c2m += e;
      }
      *reinterpret_cast<float4*>(S.r + p) = make_float4(rr[0], rr[1], rr[2], rr[3]);
      if (S.model) {
        float* mo = S.model + p;
        if ((reinterpret_cast<uintptr_t>(mo) & 15) == 0) {
          *reinterpret_cast<float4*>(mo) = make_float4(acc[0], acc[1], acc[2], acc[3]);
        } else {
          mo[0] = acc[0]; mo[1] = acc[1]; mo[2] = acc[2]; mo[3] = acc[3];
        }
      }
    }
  } else if (gi < N) {
    for (int q = 0; q < 4; ++q) {
      const int gj = tx0 + lx + q;
      if (gj >= N) break;
      const size_t p = (size_t)b * N * N + gi * N + gj;
      if (adjoint) {
        S.ubar[p] = acc[q];
      } else {
        const int pi = gi * N + gj;
        const float res = acc[q] - S.image[pi];
        const float iv = S.inv_var[pi];
        S.r[p] = res * iv;
        if (S.model) S.model[p] = acc[q];
        const double e = (double)res * (double)res * (double)iv;
        c2 += e;
        if (S.mask[pi]) c2m += e;
      }
    }
  }
  if (!adjoint) {
    double v[2] = {c2, c2m};
    block_sum<2>(v, red);
    if (threadIdx.x == 0) {
      double* o = S.c2part + ((size_t)b * S.psf_tiles + tile) * 2;
      o[0] = v[0];
      o[1] = v[1];
    }
  }
}

// The input tile with its halo (zero outside the image), then nw weights
// from W right after it, in one pass of batched loads.
__device__ __forceinline__ void psf_load_tile(const SysDev& S, int b, int adjoint, int KP, int ty0, int tx0,
                                              float* tilein, const float* W, int nw) {
  const int N = S.n_img, h = KP / 2;
  const int HW = PSF_TW + KP - 1, LS = psf_row_stride(KP), HH = PSF_TH + KP - 1;
  const int nt = HH * LS;
  const float* in = (adjoint ? S.r : S.u) + (size_t)b * N * N;
  batched_copy<8>(nt + nw,
                  [&](int q) {
                    if (q >= nt) return W[q - nt];
                    const int rr = q / LS, cc = q - rr * LS;
                    const int gi = ty0 + rr - h, gj = tx0 + cc - h;
                    return (cc < HW && gi >= 0 && gi < N && gj >= 0 && gj < N) ? in[gi * N + gj] : 0.f;
                  },
                  [&](int q, float v) { tilein[q] = v; });
  __syncthreads();
}

// out[i, j] = sum_{a,b} W[a, b] in[i + a - h, j + b - h] (zero outside), h = (KP-1)/2.
// Forward: in = u, W = flipped PSF (a convolution), also r = (m - d)/sigma^2 and
// chi^2 partials.  Adjoint: in = r, W = PSF (the transpose of the convolution).
// Wave w of the workgroup computes the 16 x 16 outputs of tile columns
// [16 w, 16 w + 16); a wave wholly right of the image skips its products.
// Lane l: A = Wp[a][4 q + l / 16 - l % 16 + 15], B = in[l % 16 + a][16 w + 4 q + l / 16];
// the accumulator holds row l % 16, columns 16 w + 4 (l / 16) + r, r < 4.
// KPT = 0: the PSF size is a run-time value.
template <int KPT>
__device__ void psf_body(const SysDev& S, int b, int tile, int adjoint, float* tilein, double* red) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const int KP = KPT ? KPT : S.psf_k;
  const int NK = psf_nk(KP), WS = psf_ws(KP), LS = psf_row_stride(KP);
  const int ty0 = (tile / S.psf_tx) * PSF_TH, tx0 = (tile % S.psf_tx) * PSF_TW;
  const float* wp = tilein + (PSF_TH + KP - 1) * LS;   // the padded weight rows
  psf_load_tile(S, b, adjoint, KP, ty0, tx0, tilein, adjoint ? S.psf : S.psf_flip, KP * WS);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  if (tx0 + wave * 16 < S.n_img) {
    const float* ap = wp + 15 + lq - lr;
    const float* bp = tilein + lr * LS + wave * 16 + lq;
    const int nk = KPT ? psf_nk(KPT) : NK;   // a constant for the templated sizes
    int a = 0;
    for (; a + 1 < KP; a += 2) {
#pragma unroll
      for (int q = 0; q < nk; ++q) {
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ap[a * WS + 4 * q], bp[a * LS + 4 * q], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ap[(a + 1) * WS + 4 * q], bp[(a + 1) * LS + 4 * q], acc1, 0,
                                                    0, 0);
      }
    }
    if (a < KP)
      for (int q = 0; q < nk; ++q)
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ap[a * WS + 4 * q], bp[a * LS + 4 * q], acc0, 0, 0, 0);
  }
  const float out[4] = {acc0[0] + acc1[0], acc0[1] + acc1[1], acc0[2] + acc1[2], acc0[3] + acc1[3]};
  psf_epilogue(S, b, tile, adjoint, ty0, tx0, lr, wave * 16 + lq * 4, out, red);
}

// A rank-one PSF, W[a][c] = u[a] v[c] (a Gaussian is one): a pass along the
// rows of the input tile with v into LDS (the tile's rows and its halo rows),
// then a pass along the columns with u; 2 K_psf instead of K_psf^2
// multiply-adds per pixel, FP32.  Each thread sums 4 consecutive columns.
template <int KPT>
__device__ void psf_sep_body(const SysDev& S, int b, int tile, int adjoint, float* tilein, double* red) {
  const int KP = KPT ? KPT : S.psf_k;
  const int N = S.n_img, LS = psf_sep_stride(KP), HH = PSF_TH + KP - 1, h = KP / 2;
  const int ty0 = (tile / S.psf_tx) * PSF_TH, tx0 = (tile % S.psf_tx) * PSF_TW;
  // the tile's rows from column tx0 - h - sh (a multiple of 4): with N a
  // multiple of 4 every row is read in aligned float4 groups, each wholly
  // inside or wholly outside the image
  const int sh = (4 - (h & 3)) & 3, gj0 = tx0 - h - sh, nq = LS / 4;
  const float* in = (adjoint ? S.r : S.u) + (size_t)b * N * N;
  if ((N & 3) == 0) {
    batched_copy<4>(HH * nq,
                    [&](int q) {
                      const int rr = q / nq, gi = ty0 + rr - h, gj = gj0 + 4 * (q - rr * nq);
                      return (gi >= 0 && gi < N && gj >= 0 && gj < N)
                                 ? *reinterpret_cast<const float4*>(in + gi * N + gj)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
                    },
                    [&](int q, float4 v) { reinterpret_cast<float4*>(tilein)[q] = v; });
  } else {
    batched_copy<8>(HH * LS,
                    [&](int q) {
                      const int rr = q / LS, gi = ty0 + rr - h, gj = gj0 + q - rr * LS;
                      return (gi >= 0 && gi < N && gj >= 0 && gj < N) ? in[gi * N + gj] : 0.f;
                    },
                    [&](int q, float v) { tilein[q] = v; });
  }
  const float* W = S.psf_sep + (adjoint ? 2 * KP : 0);
  for (int k = threadIdx.x; k < 2 * KP; k += blockDim.x) tilein[HH * LS + k] = W[k];
  __syncthreads();
  const float* uf = tilein + HH * LS;
  const float* vf = uf + KP;
  float* tr = tilein + HH * LS + ((2 * KP + 3) & ~3);    // [HH][PSF_TW] row-pass sums
  for (int it = threadIdx.x; it < HH * (PSF_TW / 4); it += blockDim.x) {
    const int rr = it / (PSF_TW / 4), x = (it - rr * (PSF_TW / 4)) * 4;
    if (tx0 + x >= S.n_img) continue;
    const float* row = tilein + rr * LS + x + sh;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
    for (int c = 0; c < (KPT ? KPT : 1); ++c) {
      if (!KPT) break;
      const float w = vf[c];
      a0 = fmaf(w, row[c], a0); a1 = fmaf(w, row[c + 1], a1); a2 = fmaf(w, row[c + 2], a2); a3 = fmaf(w, row[c + 3], a3);
    }
    if (!KPT)
      for (int c = 0; c < KP; ++c) {
        const float w = vf[c];
        a0 = fmaf(w, row[c], a0); a1 = fmaf(w, row[c + 1], a1); a2 = fmaf(w, row[c + 2], a2); a3 = fmaf(w, row[c + 3], a3);
      }
    *reinterpret_cast<float4*>(tr + rr * PSF_TW + x) = make_float4(a0, a1, a2, a3);
  }
  __syncthreads();
  const int ly = threadIdx.x >> 4, lx = (threadIdx.x & 15) * 4;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  if (tx0 + lx < S.n_img) {
    const float* col = tr + ly * PSF_TW + lx;
    for (int a = 0; a < KP; ++a) {
      const float w = uf[a];
      const float4 t = *reinterpret_cast<const float4*>(col + a * PSF_TW);
      acc[0] = fmaf(w, t.x, acc[0]); acc[1] = fmaf(w, t.y, acc[1]);
      acc[2] = fmaf(w, t.z, acc[2]); acc[3] = fmaf(w, t.w, acc[3]);
    }
  }
  psf_epilogue(S, b, tile, adjoint, ty0, tx0, ly, lx, acc, red);
}

__device__ __forceinline__ void psf_dispatch(const SysDev& S, int b, int tile, int adjoint, float* tilein,
                                             double* red) {
  if (obs_rank1(S)) {
    switch (S.psf_k) {
      case 15: psf_sep_body<15>(S, b, tile, adjoint, tilein, red); break;
      case 21: psf_sep_body<21>(S, b, tile, adjoint, tilein, red); break;
      case 31: psf_sep_body<31>(S, b, tile, adjoint, tilein, red); break;
      default: psf_sep_body<0>(S, b, tile, adjoint, tilein, red);
    }
    return;
  }
  switch (S.psf_k) {
    case 15: psf_body<15>(S, b, tile, adjoint, tilein, red); break;
    case 21: psf_body<21>(S, b, tile, adjoint, tilein, red); break;
    case 31: psf_body<31>(S, b, tile, adjoint, tilein, red); break;
    default: psf_body<0>(S, b, tile, adjoint, tilein, red);
  }
}

// Workgroup i of a launch of G is dispatched to XCD i mod 8.  This maps the
// workgroups of XCD x to one contiguous range of the G work items (XCDs
// below G mod 8 take one item more), so that neighbouring PSF tiles, whose
// input halos overlap, read them through the same L2.  A bijection on [0, G).
__device__ __forceinline__ int xcd_contiguous(int i, int G) {
  const int x = i & 7, k = i >> 3, q = G >> 3, r = G & 7;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__global__ void __launch_bounds__(PSF_THREADS) k_psf(SysDev S, int adjoint) {
  extern __shared__ __align__(16) float tilein[];
  __shared__ double red[2 * 4];
  const int w = xcd_contiguous(blockIdx.x, gridDim.x);
  const int b = w / S.psf_tiles;
  psf_dispatch(S, b, w - b * S.psf_tiles, adjoint, tilein, red);
}

// ====================================================================== k_post
// The GP adjoint's pointwise steps (eqs. 1-4), shared by the one-workgroup
// transform and the split line passes; the spectrum-parameter sums go into
// pacc (sigma, n, zeta, alpha).
struct GpAdj {
  Matern mt;
  float alpha, inv_n2, inv_sig, inv_zeta, dn_c;
  int n;
  __device__ __forceinline__ GpAdj(const float* ps, int n_) : mt(make_matern(ps)), alpha(ps[3]), n(n_) {
    inv_n2 = 1.f / (float)(n * n);
    inv_sig = 1.f / ps[0];
    inv_zeta = 1.f / mt.zeta;
    dn_c = (mt.n + 1.f) / (2.f * mt.n);
  }
  // fbar = sbar ds/df, ds/df = alpha s sigmoid(x)/(s0 softplus(x)), x = f/s0
  __device__ __forceinline__ float fbar(float sbq, float f, float s, double (&pacc)[4]) const {
    const SoftplusTerms sp = softplus_terms(f * 100.f);
    pacc[3] += (double)(sbq * s * (-4.605170186f + sp.lsp));
    return sbq * alpha * s * sp.ratio * 100.f;
  }
  // the spectrum: Re(F conj(Fbar)) sqrt(P) / n^2 times d log sqrt(P) / d (sigma, n, zeta):
  //   1/sigma,  ((n+1)/(2n)) k^2/(a+k^2) + log(a/(a+k^2))/2,  (a - n k^2)/(zeta (a+k^2));
  // returns Fbar sqrt(P)
  __device__ __forceinline__ float2 spectrum(int r, int c, float2 v, float2 f0, double (&pacc)[4]) const {
    const float kx = fft_freq(c, n), ky = fft_freq(r, n);
    const float k2 = kx * kx + ky * ky;
    const float sq = matern_sqrtP(mt, k2);
    const float re = (f0.x * v.x + f0.y * v.y) * inv_n2 * sq;
    const float iapk = 1.f / (mt.a + k2);
    pacc[0] += (double)(re * inv_sig);
    pacc[1] += (double)(re * (dn_c * k2 * iapk + 0.5f * __logf(mt.a * iapk)));
    pacc[2] += (double)(re * ((mt.a - mt.n * k2) * iapk * inv_zeta));
    return make_float2(v.x * sq, v.y * sq);
  }
};

// ====================================================================== split GP transforms
// Grids of at least GP_SPLIT_N per side: the 2-D transforms of the GP source
// (prep) and of its adjoint (post) as three line passes through the
// workspace T, each a launch of GP_LINES lines per workgroup, so that a
// sample's transform is spread over n / GP_LINES workgroups:
//   prep:    rows: T = DFT_x(w); columns: F = DFT_y(T), T = IDFT_y(sqrt(P) F);
//            rows: f = Re IDFT_x(T) / n^2, then the source;
//   adjoint: rows: T = DFT_x(fbar); columns: Fbar = DFT_y(T) with the
//            spectrum sums, T = IDFT_y(sqrt(P) Fbar); rows: d loss / d w =
//            Re IDFT_x(T) / n^2 + w.
// The adjoint's spectrum sums are kept per workgroup (gpp) and added in
// workgroup order by the last pass's first workgroup.
template <bool ADJ>
__device__ void gp_pass(const SysDev& S, int b, int pass, int part, unsigned char* smem, double* red) {
  float2* lds = reinterpret_cast<float2*>(smem);
  const int n = S.n_src, logn = S.log2_src, n2 = n * n;
  const int cap = GP_LINES * (n + 1), l0 = part * GP_LINES, l1 = l0 + GP_LINES;
  const int G = n / GP_LINES;
  float2* T = S.tmp + (size_t)b * n2;
  const float* ps = S.ps + (size_t)b * 4;
  const float* w = S.latent + (size_t)b * n2;
  auto same = [](int, int, float2 v) { return v; };
  auto to_T = [&](int r, int c, float2 v) { T[r * n + c] = v; };
  auto from_T = [&](int r, int c) { return T[r * n + c]; };
  if (!ADJ) {
    const Matern mt = make_matern(ps);
    const float alpha = ps[3], inv_n2 = 1.f / (float)n2;
    float2* F = S.F + (size_t)b * n2;
    if (pass == 0)
      fft_pass(lds, cap, n, logn, false, -1.f, false, 0.f, [&](int r, int c) { return make_float2(w[r * n + c], 0.f); },
               same, to_T, l0, l1);
    else if (pass == 1)
      fft_pass(lds, cap, n, logn, true, -1.f, true, 1.f, from_T,
               [&](int r, int c, float2 v) {
                 F[r * n + c] = v;
                 const float kx = fft_freq(c, n), ky = fft_freq(r, n);
                 const float sq = matern_sqrtP(mt, kx * kx + ky * ky);
                 return make_float2(v.x * sq, v.y * sq);
               },
               to_T, l0, l1);
    else
      fft_pass(lds, cap, n, logn, false, 1.f, false, 0.f, from_T, same,
               [&](int r, int c, float2 v) { gp_source(S, b, r * n + c, v.x * inv_n2, alpha); }, l0, l1);
    return;
  }
  const GpAdj ga(ps, n);
  double pacc[4] = {0.0, 0.0, 0.0, 0.0};
  double* gp = S.gpp + (size_t)b * (n / GP_LINES + 1) * 4;
  if (pass == 0) {
    const double* sb = S.sbar + (size_t)b * n2;
    const float* fo = S.fld + (size_t)b * n2;
    const float* so = S.src + (size_t)b * n2;
    fft_pass<2>(lds, cap, n, logn, false, -1.f, false, 0.f,
                [&](int r, int c) {
                  const int q = r * n + c;
                  return make_float2(ga.fbar((float)sb[q], fo[q], so[q], pacc), 0.f);
                },
                same, to_T, l0, l1);
    block_sum<4>(pacc, red);
    if (threadIdx.x == 0) gp[part * 4 + 3] = pacc[3];
  } else if (pass == 1) {
    const float2* F = S.F + (size_t)b * n2;
    fft_pass<2>(lds, cap, n, logn, true, -1.f, true, 1.f, from_T,
                [&](int r, int c, float2 v) { return ga.spectrum(r, c, v, F[r * n + c], pacc); }, to_T, l0, l1);
    block_sum<4>(pacc, red);
    if (threadIdx.x < 3) gp[part * 4 + threadIdx.x] = pacc[threadIdx.x];
  } else {
    uint32_t bad = 0;
    fft_pass<2>(lds, cap, n, logn, false, 1.f, false, 0.f, from_T, same,
                [&](int r, int c, float2 v) {
                  const int q = r * n + c;
                  const float g = v.x * ga.inv_n2 + w[q];
                  if (S.g_lat) S.g_lat[(size_t)b * n2 + q] = g;
                  if (!isfinite(g)) bad = 1;
                },
                l0, l1);
    if (bad) atomicOr(&S.status[b], RTU_ST_NONFINITE);
    if (part == 0 && threadIdx.x < 4) {
      double v = 0.0;
      for (int g = 0; g < G; ++g) v += gp[g * 4 + threadIdx.x];
      if (S.g_ps) S.g_ps[(size_t)b * 4 + threadIdx.x] = (float)v;
      if (!isfinite(v)) atomicOr(&S.status[b], RTU_ST_NONFINITE);
    }
  }
}

template <bool ADJ>
__global__ void __launch_bounds__(GP_THREADS) k_gp(SysDev S, int pass) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[4 * (GP_THREADS / 64)];
  if (ADJ && !S.want_grad) return;
  const int G = S.n_src / GP_LINES;
  const int b = blockIdx.x / G;
  gp_pass<ADJ>(S, b, pass, blockIdx.x - b * G, smem, red);
}

struct PostLds {
  double red[16 * 16];
  double part[POST_THREADS];
  double xbar[2][K];      // d loss / d X (beta units), after the slope chain
  double wk[2][K];        // -S_k^2 d loss / d S_k
  double lsum[RTU_MAX_LENS + 1];   // raw sums
  double ub[4];           // uniform grid: d loss / d (x_min, x_max, y_min, y_max)
  uint32_t stat;
  EplTab etab;            // EPL deflector: the sample's series tables
};

__device__ __forceinline__ void post_body(const SysDev& S, int b, int role, unsigned char* fft_smem, int cap, PostLds& P) {
  const int tid = threadIdx.x;
  const int n = S.n_src, n2 = n * n, logn = S.log2_src;
  const int nl = S.n_lens;
  if (tid == 0) P.stat = 0;
  __syncthreads();
  // ---- role 0: loss and chi^2 in the mask, then the lens gradient
  if (role == 0) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = tid; t < S.psf_tiles; t += blockDim.x) {
      const double* o = S.c2part + ((size_t)b * S.psf_tiles + t) * 2;
      v[0] += o[0];
      v[1] += o[1];
    }
    const float* w = S.latent + (size_t)b * n2;
    batched_copy<8>(n2, [&](int q) { return w[q]; }, [&](int, float x) { v[2] += (double)x * x; });
    block_sum<3>(v, P.red);
    if (tid == 0) {
      const double loss = 0.5 * v[0] + 0.5 * v[2];
      S.loss[b] = loss;
      const int M = obs_M(S);
      if (S.chi2m) S.chi2m[b] = M > 0 ? v[1] / (double)M : 0.0;
      if (!isfinite(loss)) P.stat |= RTU_ST_NONFINITE;
    }
  }
  if (role == 0 && S.want_grad) {
    const float* lensp = S.lens + (size_t)b * nl;
    const int nsub = n_sub_of(S, b);
    const Sie L = S.epl ? make_sie(lensp) : S.sie[b];   // (the EPL path does not use it)
    if (S.epl && tid == 0) epl_table(make_epl(lensp), P.etab);   // read after the syncs below
    // ---- knot adjoint: sum the tile partials, then S_k = 1/p'_k with
    //      p'_k = sum_l D_kl X_l  ->  dX_l += sum_k (-S_k^2 dS_k) D_kl
    reduce_columns(S.kbar + (size_t)b * S.ray_tiles * 4 * K, S.ray_tiles, 4 * K, 4 * K,
                   P.part, [&](int c, double v) { P.red[c] = v; });
    __syncthreads();
    // the factors -S_k^2 dS_k, one thread per (axis, k); then the sums over k
    if (!S.uniform && tid < 2 * K) {
      const int ax = tid / K, k = tid - ax * K;
      const double d = S.dp[((size_t)b * 2 + ax) * K + k];
      P.wk[ax][k] = d > 0.0 ? -P.red[ax * 2 * K + K + k] / (d * d) : 0.0;
    }
    // uniform grid: y = (beta - lo) / L with the moment sums m0 = sum ybar,
    // m1 = sum ybar y per axis gives d/d lo_a = -m0_a / L and
    // d/d L = -(m1_x + m1_y) / L; lo_a = (min_a + max_a)/2 - L/2 and L the
    // longer range (x on a tie) carry them to the four extremes.  A
    // degenerate box (status bit 4) is a constant.
    if (S.uniform && tid == 0) {
      const double* sd = S.stdv + (size_t)b * 4;
      const double side = sd[2];
      const bool degen = (S.st[b * ST_WORDS] & RTU_ST_MASK_SMALL) != 0;
      const double glo[2] = {-P.red[0] / side, -P.red[2 * K] / side};
      const double gL = -(P.red[1] + P.red[2 * K + 1]) / side;
      const double gc = gL - 0.5 * (glo[0] + glo[1]);
      const int lax = (int)sd[3];   // the axis whose range is L
      for (int a = 0; a < 2; ++a) {
        const double dl = a == lax ? 1.0 : 0.0;
        P.ub[2 * a] = degen ? 0.0 : 0.5 * glo[a] - gc * dl;
        P.ub[2 * a + 1] = degen ? 0.0 : 0.5 * glo[a] + gc * dl;
      }
    }
    __syncthreads();
    if (!S.uniform && tid < 2 * K) {
      const int ax = tid / K, l = tid - ax * K;
      double xb = P.red[ax * 2 * K + l];
#pragma unroll
      for (int k = 0; k < K; ++k) xb += P.wk[ax][k] * c_D[k * K + l];
      P.xbar[ax][l] = xb;
    }
    __syncthreads();
    // ---- selected masked rays: X_k = (1-t_k) beta_(j) + t_k beta_(j+1); each of
    //      the 4K (axis, rank) items writes its lens-gradient row into LDS
    const int nc = nl + 1;   // raw SIE + shear accumulators (8), subhalo terms
    double* mp = reinterpret_cast<double*>(fft_smem);   // [4K][nc]
    if (tid < 4 * K) {
      double* row = mp + tid * nc;
      for (int q = 0; q < nc; ++q) row[q] = 0.0;
      int ax, m;
      double bb;
      if (S.uniform) {   // rows 0..3: the minimum and maximum of x, then of y
        ax = (tid >> 1) & 1;
        m = S.sel[((size_t)b * 2 + ax) * 2 * K + (tid & 1)];
        bb = tid < 4 ? P.ub[tid] : 0.0;
      } else {
        ax = tid / (2 * K);
        const int r = tid - ax * 2 * K, k = r >> 1;
        const double t = S.ray_w ? S.wt[k] : S.rank_t[k];
        const double wgt = (r & 1) ? t : 1.0 - t;
        m = S.sel[((size_t)b * 2 + ax) * 2 * K + r];
        bb = wgt * P.xbar[ax][k];
      }
      const int M = obs_M(S);
      m = m < 0 ? 0 : (m >= M ? M - 1 : m);
      if (bb != 0.0 && M > 0) {
        const float2 c = S.mask_xy[m];
        const float x = c.x, y = c.y;
        const float abx = ax == 0 ? -(float)bb : 0.f, aby = ax == 1 ? -(float)bb : 0.f;
        if (S.epl) {     // the parameter gradients themselves (row 8 stays zero)
          float ea[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
          epl_shear_vjp(make_epl(lensp), P.etab, x, y, abx, aby, ea);
          for (int k = 0; k < 8; ++k) row[k] = ea[k];
        } else {
          SieAcc a;
          a.zero();
          SieRay E;
          float ax_, ay_;
          sie_shear_alpha<true>(L, x, y, ax_, ay_, E);
          sie_shear_vjp(L, E, x, y, abx, aby, a);
          row[0] = a.P; row[1] = a.q; row[2] = a.f; row[3] = a.phi;
          row[4] = a.x0; row[5] = a.y0; row[6] = a.g1; row[7] = a.g2;
        }
        double* rs = row + S.lens_base + 1;   // lens index + 1 from the subhaloes on
        for (int q = 0; q < nsub; ++q) {
          const Nfw N = make_nfw(lensp + S.lens_base + RTU_N_PER_SUB * q, S.tau);
          float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f;
          nfw_vjp(N, S.tau, x, y, abx, aby, g0, g1, g2, g3);
          rs[4 * q] = g0; rs[4 * q + 1] = g1; rs[4 * q + 2] = g2; rs[4 * q + 3] = g3;
        }
      }
    }
    __syncthreads();
    // the per-wave tile rows, then the masked-ray rows, each summed in a
    // fixed order; then the chain from the SIE quantities to the lens
    // parameters, once
    const int rows = S.ray_tiles * (RAY_THREADS / 64);
    reduce_columns(S.lpart + (size_t)b * rows * (nc + 1), rows, nc, nc + 1, P.part,
                   [&](int c, double v) { P.lsum[c] = v; });
    __syncthreads();
    reduce_columns(mp, 4 * K, nc, nc, P.part, [&](int c, double v) { P.lsum[c] += v; });
    __syncthreads();
    if (tid < nl) {
      const double v = S.epl ? (tid < 8 ? P.lsum[tid] : P.lsum[tid + 1])
                             : (tid < 7 ? sie_grad_one(L, P.lsum, tid) : P.lsum[tid + 1]);
      if (S.g_lens) S.g_lens[(size_t)b * nl + tid] = (float)v;
      if (!isfinite(v)) atomicOr(&P.stat, RTU_ST_NONFINITE);
    }
  }
  // ---- role 1: the GP adjoint (split grids: three line-pass launches, gp_pass)
  if (role == 1 && !gp_split(n)) {
    const float* ps = S.ps + (size_t)b * 4;
    const GpAdj ga(ps, n);
    const double* sb = S.sbar + (size_t)b * n2;
    const float* fo = S.fld + (size_t)b * n2;
    const float* so = S.src + (size_t)b * n2;
    const float2* F = S.F + (size_t)b * n2;
    const float* w = S.latent + (size_t)b * n2;
    float2* lds = reinterpret_cast<float2*>(fft_smem);
    double pacc[4] = {0.0, 0.0, 0.0, 0.0};   // sigma, n, zeta, alpha
    auto fbar_of = [&](float sbq, float f, float s) { return ga.fbar(sbq, f, s, pacc); };
    auto spectrum = [&](int r, int c, float2 v, float2 f0) { return ga.spectrum(r, c, v, f0, pacc); };
    uint32_t bad = 0;
    auto latent_grad = [&](int q, float v, float wq) {
      const float g = v * ga.inv_n2 + wq;
      if (S.g_lat) S.g_lat[(size_t)b * n2 + q] = g;
      if (!isfinite(g)) bad = 1;
    };
    {
      // the whole grid in LDS (as in the prep transform; F in split layout)
      float2* tw = lds + cap;
      for (int k = tid; k < 128; k += blockDim.x) tw[k] = c_tw[k];
      const int ls = n + 1;
      // four consecutive points of a row per item (n >= 8): two double2
      // loads of d loss / d s, float4 loads of the field and the source
      struct G4 {
        double2 a, c;
        float4 f, s;
      };
      batched_copy<4>(n2 >> 2,
                      [&](int q4) {
                        G4 g;
                        g.a = reinterpret_cast<const double2*>(sb)[2 * q4];
                        g.c = reinterpret_cast<const double2*>(sb)[2 * q4 + 1];
                        g.f = reinterpret_cast<const float4*>(fo)[q4];
                        g.s = reinterpret_cast<const float4*>(so)[q4];
                        return g;
                      },
                      [&](int q4, const G4& g) {
                        float2* row = lds + ((4 * q4) >> logn) * ls + ((4 * q4) & (n - 1));
                        row[0] = make_float2(fbar_of((float)g.a.x, g.f.x, g.s.x), 0.f);
                        row[1] = make_float2(fbar_of((float)g.a.y, g.f.y, g.s.y), 0.f);
                        row[2] = make_float2(fbar_of((float)g.c.x, g.f.z, g.s.z), 0.f);
                        row[3] = make_float2(fbar_of((float)g.c.y, g.f.w, g.s.w), 0.f);
                      });
      __syncthreads();
      fft_grid_dir(lds, tw, n, logn, false, -1.f, true);
      fft_grid_dir(lds, tw, n, logn, true, -1.f, true);
      // F: four consecutive entries of a row per item (two float4 loads)
      struct F4 {
        float4 lo, hi;
      };
      batched_copy<4>(n2 >> 2,
                      [&](int q4) {
                        const float4* f4 = reinterpret_cast<const float4*>(F);
                        return F4{f4[2 * q4], f4[2 * q4 + 1]};
                      },
                      [&](int q4, const F4& g) {
                        const int rs = (4 * q4) >> logn, cs = (4 * q4) & (n - 1);
                        const int r = split_nat(rs, logn);
                        float2* a = lds + rs * ls + cs;
                        a[0] = spectrum(r, split_nat(cs, logn), a[0], make_float2(g.lo.x, g.lo.y));
                        a[1] = spectrum(r, split_nat(cs + 1, logn), a[1], make_float2(g.lo.z, g.lo.w));
                        a[2] = spectrum(r, split_nat(cs + 2, logn), a[2], make_float2(g.hi.x, g.hi.y));
                        a[3] = spectrum(r, split_nat(cs + 3, logn), a[3], make_float2(g.hi.z, g.hi.w));
                      });
      __syncthreads();
      fft_grid_dir(lds, tw, n, logn, true, 1.f, false);
      fft_grid_dir(lds, tw, n, logn, false, 1.f, false);
      batched_copy<8>(n2 >> 2, [&](int q4) { return reinterpret_cast<const float4*>(w)[q4]; },
                      [&](int q4, float4 v) {
                        const int q = 4 * q4;
                        const float2* a = lds + (q >> logn) * ls + (q & (n - 1));
                        latent_grad(q, a[0].x, v.x);
                        latent_grad(q + 1, a[1].x, v.y);
                        latent_grad(q + 2, a[2].x, v.z);
                        latent_grad(q + 3, a[3].x, v.w);
                      });
    }
    if (bad) atomicOr(&P.stat, RTU_ST_NONFINITE);
    block_sum<4>(pacc, P.red);
    if (tid < 4 && S.g_ps) {
      S.g_ps[(size_t)b * 4 + tid] = (float)pacc[tid];
      if (!isfinite(pacc[tid])) atomicOr(&P.stat, RTU_ST_NONFINITE);
    }
  }
  __syncthreads();
  // status: each role ORs its word (role 0 also the selection and domain
  // words) into the sample's status, which prep cleared
  if (tid == 0) {
    const uint32_t* st = S.st + (size_t)b * ST_WORDS;
    atomicOr(&S.status[b], role == 0 ? (P.stat | st[0] | st[1] | st[2]) : P.stat);
  }
}

__global__ void __launch_bounds__(POST_THREADS) k_post(SysDev S, int fft_cap) {
  extern __shared__ __align__(16) unsigned char fft_smem[];
  __shared__ PostLds P;
  // one inlined copy per role, so that each holds only its own code
  if (blockIdx.y == 0) post_body(S, blockIdx.x, 0, fft_smem, fft_cap, P);
  else post_body(S, blockIdx.x, 1, fft_smem, fft_cap, P);
}

// ====================================================================== k_observe
// An observation prepared on the device, for the allocation-free entry point:
// the same tables the host prepares for a plan, bit for bit.
//  - inv_var = 1/sigma^2;
//  - the PSF weight rows of the forward (flipped) and adjoint correlations,
//    zero-padded: W[a][c] at [a][c + 15] of rows of psf_ws(KP);
//  - rank-one factors: u the column and v the row (divided by the pivot, in
//    FP64) through the largest |weight| (the first in row-major order), the
//    PSF taken as rank one if every weight is reproduced to 4e-7 of the
//    largest;
//  - the masked pixels in row-major order, their count M, and the quantile
//    ranks h_k = (M - 1) u_k (FP64, floor and fraction).
// One workgroup.
constexpr int OBS_THREADS = 1024;
__global__ void __launch_bounds__(OBS_THREADS) k_observe(SysDev S, const float* __restrict__ sigma,
                                                         const float* __restrict__ psf, int* dyn) {
  __shared__ float rv[OBS_THREADS];
  __shared__ int ri[OBS_THREADS];
  __shared__ double re[OBS_THREADS];
  __shared__ int wcnt[OBS_THREADS / 64];
  __shared__ int s_off;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int N2 = S.n_img * S.n_img, KP = S.psf_k, WS = psf_ws(KP);
  float* fwd = const_cast<float*>(S.psf_flip);
  float* adj = const_cast<float*>(S.psf);
  float* sep = const_cast<float*>(S.psf_sep);
  for (int q = tid; q < KP * WS; q += OBS_THREADS) {
    const int a = q / WS, c = q - a * WS - 15;
    const bool in = c >= 0 && c < KP;
    fwd[q] = in ? psf[(KP - 1 - a) * KP + (KP - 1 - c)] : 0.f;
    adj[q] = in ? psf[a * KP + c] : 0.f;
  }
  // the largest |weight|, the first in row-major order among equal ones
  float bv = 0.f;
  int bi = 0x7fffffff;
  for (int q = tid; q < KP * KP; q += OBS_THREADS) {
    const float v = fabsf(psf[q]);
    if (v > bv) { bv = v; bi = q; }
  }
  rv[tid] = bv;
  ri[tid] = bi;
  __syncthreads();
  for (int w = OBS_THREADS / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const float v2 = rv[tid + w];
      const int i2 = ri[tid + w];
      if (v2 > rv[tid] || (v2 == rv[tid] && i2 < ri[tid])) { rv[tid] = v2; ri[tid] = i2; }
    }
    __syncthreads();
  }
  const double wmax = (double)rv[0];
  const int ar = wmax > 0.0 ? ri[0] / KP : 0, ac = wmax > 0.0 ? ri[0] - ar * KP : 0;
  const double piv = psf[ar * KP + ac];
  auto uf = [&](int a) { return psf[a * KP + ac]; };
  auto vf = [&](int c) { return (float)((double)psf[ar * KP + c] / piv); };
  double err = 0.0;
  if (wmax > 0.0)
    for (int q = tid; q < KP * KP; q += OBS_THREADS) {
      const int a = q / KP, c = q - a * KP;
      err = fmax(err, fabs((double)psf[q] - (double)uf(a) * (double)vf(c)));
    }
  re[tid] = err;
  __syncthreads();
  for (int w = OBS_THREADS / 2; w > 0; w >>= 1) {
    if (tid < w) re[tid] = fmax(re[tid], re[tid + w]);
    __syncthreads();
  }
  const int rank1 = wmax > 0.0 && re[0] <= 4e-7 * wmax;
  for (int a = tid; a < KP; a += OBS_THREADS) {
    sep[a] = wmax > 0.0 ? uf(KP - 1 - a) : 0.f;
    sep[KP + a] = wmax > 0.0 ? vf(KP - 1 - a) : 0.f;
    sep[2 * KP + a] = wmax > 0.0 ? uf(a) : 0.f;
    sep[3 * KP + a] = wmax > 0.0 ? vf(a) : 0.f;
  }
  // inverse variances and the masked pixels in row-major order (a running
  // offset over chunks of OBS_THREADS pixels, ballot ranks inside each wave)
  float* iv = const_cast<float*>(S.inv_var);
  int* idx = const_cast<int*>(S.mask_idx);
  if (tid == 0) s_off = 0;
  __syncthreads();
  for (int base = 0; base < N2; base += OBS_THREADS) {
    const int p = base + tid;
    const bool m = p < N2 && S.mask[p] != 0;
    if (p < N2) {
      const float sg = sigma[p];
      iv[p] = 1.f / (sg * sg);
    }
    const unsigned long long bal = __ballot(m);
    const int below = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wv] = __popcll(bal);
    __syncthreads();
    int off = s_off;
    for (int w = 0; w < wv; ++w) off += wcnt[w];
    if (m) {
      idx[off + below] = p;
      const_cast<float2*>(S.mask_xy)[off + below] = pixel_centre(p, S.n_img, S.pix);
    }
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int w = 0; w < OBS_THREADS / 64; ++w) t += wcnt[w];
      s_off += t;
    }
    __syncthreads();
  }
  const int M = s_off;
  if (tid < K) {
    const double hh = (double)(M > 0 ? M - 1 : 0) * c_ud[tid];
    const double fl = floor(hh);
    const_cast<int*>(S.rank_j)[tid] = (int)fl;
    const_cast<double*>(S.rank_t)[tid] = hh - fl;
  }
  if (tid == 0) {
    dyn[0] = M;
    dyn[1] = rank1;
    int rj[K];
    for (int k = 0; k < K; ++k) rj[k] = (int)floor((double)(M > 0 ? M - 1 : 0) * c_ud[k]);
    target_list(rj, M, const_cast<int*>(S.tsel));
  }
}

hipError_t launch_observe(const SysDev& h, const float* noise_sigma, const float* psf, int* dyn, hipStream_t s) {
  hipLaunchKernelGGL(k_observe, dim3(1), dim3(OBS_THREADS), 0, s, h, noise_sigma, psf, dyn);
  return hipGetLastError();
}

// ====================================================================== launchers
hipError_t configure_fft_kernels();

hipError_t upload_constants() {
  double u[K], tn[K];
  for (int k = 0; k < K; ++k) {
    u[k] = 0.5 * (1.0 - cos((2.0 * (k + 1) - 1.0) * M_PI / (2.0 * K)));
    tn[k] = 2.0 * u[k] - 1.0;
  }
  // T_j(t_l) and U_j(t_k) by recurrence
  double T[K][K], U[K][K];
  for (int k = 0; k < K; ++k) {
    T[0][k] = 1.0; T[1][k] = tn[k];
    U[0][k] = 1.0; U[1][k] = 2.0 * tn[k];
    for (int j = 2; j < K; ++j) {
      T[j][k] = 2.0 * tn[k] * T[j - 1][k] - T[j - 2][k];
      U[j][k] = 2.0 * tn[k] * U[j - 1][k] - U[j - 2][k];
    }
  }
  // p'(u_k) = 2 sum_{j>=1} j c_j U_{j-1}(t_k),  c_j = (2/K) sum_l q_l T_j(t_l)
  double D[K * K];
  for (int k = 0; k < K; ++k)
    for (int l = 0; l < K; ++l) {
      double s = 0.0;
      for (int j = 1; j < K; ++j) s += 2.0 * j * U[j - 1][k] * (2.0 / K) * T[j][l];
      D[k * K + l] = s;
    }
  float uf[K];
  for (int k = 0; k < K; ++k) uf[k] = (float)u[k];
  float2 tw[128];
  for (int k = 0; k < 128; ++k) tw[k] = make_float2((float)cos(2.0 * M_PI * k / 256.0), (float)-sin(2.0 * M_PI * k / 256.0));
  hipError_t e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_u), uf, sizeof(uf))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_ud), u, sizeof(u))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_D), D, sizeof(D))) != hipSuccess) return e;
  if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_tw), tw, sizeof(tw))) != hipSuccess) return e;
  return configure_fft_kernels();
}

// The FFT keeps min(n, cap / (n + 1)) lines of the grid in LDS at a time:
// every line of a grid up to 128 per side, 64-line chunks beyond.
// The buffer holds the lines plus the 128-entry twiddle table.
int fft_lds_cap(int n_src) { return gp_split(n_src) ? 0 : n_src * (n_src + 1); }
size_t gp_lds_bytes(int n_src) { return (size_t)(GP_LINES * (n_src + 1) + 128) * sizeof(float2); }
size_t prep_lds_bytes(int n_src) {
  const size_t f = (size_t)(fft_lds_cap(n_src) + 128) * sizeof(float2);
  return f > sizeof(SelLds) ? f : sizeof(SelLds);
}
// k_post shares its dynamic LDS between the FFT lines and the per-node
// lens-gradient rows of the masked rays ([4K][n_lens + 1] doubles).
size_t post_lds_bytes(int n_src, int n_lens) {
  const size_t f = (size_t)(fft_lds_cap(n_src) + 128) * sizeof(float2);
  const size_t m = (size_t)4 * K * (n_lens + 1) * sizeof(double);
  return f > m ? f : m;
}

hipError_t launch_prep(const SysDev& h, int batch, hipStream_t s) {
  if (h.mr_nchunk) hipLaunchKernelGGL(k_mrays, dim3(h.mr_nchunk, batch), dim3(MR_THREADS), 0, s, h);
  hipLaunchKernelGGL(k_prep, dim3(batch, 3), dim3(prep_threads(h.obs_dyn ? 0 : h.M, h.n_src)), prep_lds_bytes(h.n_src), s, h,
                     fft_lds_cap(h.n_src));
  if (gp_split(h.n_src))
    for (int pass = 0; pass < 3; ++pass)
      hipLaunchKernelGGL(k_gp<false>, dim3(batch * (h.n_src / GP_LINES)), dim3(GP_THREADS), gp_lds_bytes(h.n_src), s,
                         h, pass);
  return hipGetLastError();
}

// The ray adjoint keeps d loss / d s in LDS when the grid is at most
// GRID_LDS_MAX per side and the workgroup's LDS stays within 64 KB.
// The forward keeps only the spline tables in LDS; the adjoint also keeps
// d loss / d s (FP64) of the whole grid when it is small enough.
// The global-mode window: as many grid points as keep the adjoint within 64 KB
// of LDS, at most ADJ_WCAP_MAX (the tiles of the n = 128 workloads mostly touch
// 1-2k points).
constexpr int ADJ_WCAP_MAX = 3072;
int adj_window_cap(const SysDev& h) {
  const long fixed = (long)sizeof(RayLdsHead) + 4L * h.n_sub_max * RAY_THREADS * 4 + 16;
  const long room = (65536 - fixed) / 8;
  return (int)(std::max(0L, std::min((long)ADJ_WCAP_MAX, room)) & ~1L);
}

size_t ray_lds_bytes(const SysDev& h, bool adjoint, bool lds_grid) {
  if (!adjoint) return sizeof(RayLdsHead);
  const size_t np = (size_t)(h.n_src + 2);
  size_t bytes = sizeof(RayLdsHead) + (lds_grid ? np * np * 8 : (size_t)h.adj_wcap * 8) +
                 (size_t)4 * h.n_sub_max * RAY_THREADS * 4;
  return (bytes + 15) & ~(size_t)15;
}
bool adj_lds_grid(const SysDev& h) {
  return h.n_src <= GRID_LDS_MAX && ray_lds_bytes(h, true, true) <= 65536;
}

hipError_t launch_rays_fwd(const SysDev& h, int batch, hipStream_t s) {
  if (h.epl)
    hipLaunchKernelGGL(k_rays_fwd<true>, dim3(batch * h.ray_tiles), dim3(RAY_THREADS), ray_lds_bytes(h, false, false),
                       s, h);
  else
    hipLaunchKernelGGL(k_rays_fwd<false>, dim3(batch * h.ray_tiles), dim3(RAY_THREADS), ray_lds_bytes(h, false, false),
                       s, h);
  return hipGetLastError();
}

hipError_t launch_rays_adj(const SysDev& h, int batch, hipStream_t s) {
  const bool lg = adj_lds_grid(h);
  const size_t lds = ray_lds_bytes(h, true, lg);
  const dim3 g(batch * h.ray_tiles), t(RAY_THREADS);
  if (h.n_sub_max > 0) {   // subhaloes: the variant that keeps their terms in registers
    if (lg && h.epl) hipLaunchKernelGGL((k_rays_adj_sub<true, true>), g, t, lds, s, h);
    else if (lg) hipLaunchKernelGGL((k_rays_adj_sub<true, false>), g, t, lds, s, h);
    else if (h.epl) hipLaunchKernelGGL((k_rays_adj_sub<false, true>), g, t, lds, s, h);
    else hipLaunchKernelGGL((k_rays_adj_sub<false, false>), g, t, lds, s, h);
  } else if (lg && h.epl) hipLaunchKernelGGL((k_rays_adj<true, true>), g, t, lds, s, h);
  else if (lg) hipLaunchKernelGGL((k_rays_adj<true, false>), g, t, lds, s, h);
  else if (h.epl) hipLaunchKernelGGL((k_rays_adj<false, true>), g, t, lds, s, h);
  else hipLaunchKernelGGL((k_rays_adj<false, false>), g, t, lds, s, h);
  return hipGetLastError();
}

// input tile, then the zero-padded weight rows (matrix-core kernel) or the
// rank-one factors and the row-pass sums (separable kernel)
size_t psf_lds_bytes(int KP) {
  const size_t tile = (size_t)(PSF_TH + KP - 1) * psf_row_stride(KP);
  const size_t mfma = tile + (size_t)KP * psf_ws(KP);
  const size_t sep = (size_t)(PSF_TH + KP - 1) * psf_sep_stride(KP) + (size_t)((2 * KP + 3) & ~3) +
                     (size_t)(PSF_TH + KP - 1) * PSF_TW;
  return (mfma > sep ? mfma : sep) * 4;
}

hipError_t launch_psf(const SysDev& h, int batch, bool adjoint, hipStream_t s) {
  hipLaunchKernelGGL(k_psf, dim3(batch * h.psf_tiles), dim3(PSF_THREADS), psf_lds_bytes(h.psf_k), s, h,
                     adjoint ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_post(const SysDev& h, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_post, dim3(batch, h.want_grad ? 2 : 1), dim3(POST_THREADS), post_lds_bytes(h.n_src, h.n_lens), s, h,
                     fft_lds_cap(h.n_src));
  if (h.want_grad && gp_split(h.n_src))
    for (int pass = 0; pass < 3; ++pass)
      hipLaunchKernelGGL(k_gp<true>, dim3(batch * (h.n_src / GP_LINES)), dim3(GP_THREADS), gp_lds_bytes(h.n_src), s,
                         h, pass);
  return hipGetLastError();
}


// ====================================================================== shared launches
// Serving: every work item names its system; systems outside their step
// window skip.  The bodies are the ones of the single-system kernels.
__device__ __forceinline__ bool sys_active(const SysDev& S, int round) {
  const int st = round - S.round0;
  return st >= 0 && st < S.nsteps;
}

__global__ void __launch_bounds__(PREP_THREADS_WIDE) kf_prep(const SysDev* __restrict__ sys, const Task* __restrict__ tasks,
                                                      int round, int fft_cap) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Task t = tasks[blockIdx.x];
  const SysDev S = sys[t.x];
  if (!sys_active(S, round)) return;
  if (t.z < 2) prep_select(S, t.y, t.z, smem);
  else prep_gp(S, t.y, smem, fft_cap);
}

__global__ void __launch_bounds__(MR_THREADS) kf_mrays(const SysDev* __restrict__ sys, const Task* __restrict__ tasks,
                                                     int round) {
  __shared__ MRayLds L;
  const Task t = tasks[blockIdx.x];
  const SysDev S = sys[t.x];
  if (!sys_active(S, round)) return;
  mrays_body(S, t.y, t.z, L);
}

template <bool ADJ>
__global__ void __launch_bounds__(GP_THREADS) kf_gp(const SysDev* __restrict__ sys, const Task* __restrict__ tasks,
                                                    int round, int pass) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[4 * (GP_THREADS / 64)];
  const Task t = tasks[blockIdx.x];
  const SysDev S = sys[t.x];
  if (!sys_active(S, round) || (ADJ && !S.want_grad)) return;
  gp_pass<ADJ>(S, t.y, pass, t.z, smem, red);
}

template <bool EPL>
__global__ void __launch_bounds__(RAY_THREADS) kf_rays_fwd(const SysDev* __restrict__ sys,
                                                           const Task* __restrict__ tasks, int round) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Task t = tasks[blockIdx.x];
  const SysDev S = sys[t.x];
  if (!sys_active(S, round)) return;
  rays_fwd_body<EPL>(S, t.y, t.z, smem);
}

template <bool LDSGRID, bool EPL>
__global__ void __launch_bounds__(RAY_THREADS) kf_rays_adj(const SysDev* __restrict__ sys,
                                                           const Task* __restrict__ tasks, int round) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Task t = tasks[blockIdx.x];
  const SysDev S = sys[t.x];
  if (!sys_active(S, round)) return;
  rays_adj_body<LDSGRID, EPL>(S, t.y, t.z, smem);
}
template <bool LDSGRID, bool EPL>
__global__ void __launch_bounds__(RAY_THREADS) kf_rays_adj_sub(const SysDev* __restrict__ sys,
                                                               const Task* __restrict__ tasks, int round) {
  extern __shared__ __align__(16) unsigned char smem[];
  const Task t = tasks[blockIdx.x];
  const SysDev S = sys[t.x];
  if (!sys_active(S, round)) return;
  rays_adj_body<LDSGRID, EPL, true>(S, t.y, t.z, smem);
}

__global__ void __launch_bounds__(PSF_THREADS) kf_psf(const SysDev* __restrict__ sys, const Task* __restrict__ tasks,
                                                    int round, int adjoint) {
  extern __shared__ __align__(16) float tilein[];
  __shared__ double red[2 * 4];
  const Task t = tasks[xcd_contiguous(blockIdx.x, gridDim.x)];
  const SysDev S = sys[t.x];
  if (!sys_active(S, round)) return;
  psf_dispatch(S, t.y, t.z, adjoint, tilein, red);
}

__global__ void __launch_bounds__(POST_THREADS) kf_post(const SysDev* __restrict__ sys, const Task* __restrict__ tasks,
                                                      int round, int fft_cap) {
  extern __shared__ __align__(16) unsigned char fft_smem[];
  __shared__ PostLds P;
  const Task t = tasks[blockIdx.x];
  const SysDev S = sys[t.x];
  if (!sys_active(S, round)) return;
  if (t.z == 0) post_body(S, t.y, 0, fft_smem, fft_cap, P);
  else post_body(S, t.y, 1, fft_smem, fft_cap, P);
}

hipError_t launch_fleet_fit_stage(const FleetLaunch& L, int stage, int round, const float* eps, hipStream_t s);

hipError_t launch_fleet_stage(const FleetLaunch& L, int stage, int round, const float* eps, hipStream_t s) {
  switch (stage) {
    case RTU_STAGE_PREP:
      if (L.n_mr)
        hipLaunchKernelGGL(kf_mrays, dim3(L.n_mr), dim3(MR_THREADS), 0, s, L.sys, L.t_mr, round);
      if (L.n_prep)
        hipLaunchKernelGGL(kf_prep, dim3(L.n_prep), dim3(L.prep_threads), L.lds_prep, s, L.sys, L.t_prep, round,
                           (int)(L.lds_prep / sizeof(float2)) - 128);
      if (L.n_gp)
        for (int pass = 0; pass < 3; ++pass)
          hipLaunchKernelGGL(kf_gp<false>, dim3(L.n_gp), dim3(GP_THREADS), L.lds_gp, s, L.sys, L.t_gp, round, pass);
      break;
    case RTU_STAGE_RAYS_FWD:
      if (L.n_fwd[0])
        hipLaunchKernelGGL(kf_rays_fwd<false>, dim3(L.n_fwd[0]), dim3(RAY_THREADS), L.lds_rays_fwd, s, L.sys,
                           L.t_fwd[0], round);
      if (L.n_fwd[1])
        hipLaunchKernelGGL(kf_rays_fwd<true>, dim3(L.n_fwd[1]), dim3(RAY_THREADS), L.lds_rays_fwd, s, L.sys,
                           L.t_fwd[1], round);
      break;
    case RTU_STAGE_PSF_FWD:
    case RTU_STAGE_PSF_ADJ:
      if (L.n_psf)
        hipLaunchKernelGGL(kf_psf, dim3(L.n_psf), dim3(PSF_THREADS), L.lds_psf, s, L.sys, L.t_psf, round,
                           stage == RTU_STAGE_PSF_ADJ ? 1 : 0);
      break;
    case RTU_STAGE_RAYS_ADJ:
      // lists with a system that has subhaloes take the variant that keeps
      // their terms in registers
#define RTU_ADJ_LAUNCH(G, E)                                                                              \
      if (L.n_adj[G ? 0 : 1][E]) {                                                                        \
        if (L.adj_sub[G ? 0 : 1][E])                                                                      \
          hipLaunchKernelGGL((kf_rays_adj_sub<G, E>), dim3(L.n_adj[G ? 0 : 1][E]), dim3(RAY_THREADS),     \
                             L.lds_rays_adj, s, L.sys, L.t_adj[G ? 0 : 1][E], round);                     \
        else                                                                                              \
          hipLaunchKernelGGL((kf_rays_adj<G, E>), dim3(L.n_adj[G ? 0 : 1][E]), dim3(RAY_THREADS),         \
                             L.lds_rays_adj, s, L.sys, L.t_adj[G ? 0 : 1][E], round);                     \
      }
      RTU_ADJ_LAUNCH(true, false)
      RTU_ADJ_LAUNCH(true, true)
      RTU_ADJ_LAUNCH(false, false)
      RTU_ADJ_LAUNCH(false, true)
#undef RTU_ADJ_LAUNCH
      break;
    case RTU_STAGE_POST:
      if (L.n_post)
        hipLaunchKernelGGL(kf_post, dim3(L.n_post), dim3(POST_THREADS), L.lds_post, s, L.sys, L.t_post, round,
                           (int)(L.lds_post / sizeof(float2)) - 128);
      if (L.n_gp)
        for (int pass = 0; pass < 3; ++pass)
          hipLaunchKernelGGL(kf_gp<true>, dim3(L.n_gp), dim3(GP_THREADS), L.lds_gp, s, L.sys, L.t_gp, round, pass);
      break;
    default:
      return launch_fleet_fit_stage(L, stage, round, eps, s);
  }
  return hipGetLastError();
}

// The FFT kernels may take up to 129 KB of dynamic LDS (plus their static
// part) of the 160 KB per CU.
hipError_t configure_fft_kernels() {
  const int big = (int)(prep_lds_bytes(128) > post_lds_bytes(128, RTU_MAX_LENS) ? prep_lds_bytes(128)
                                                                               : post_lds_bytes(128, RTU_MAX_LENS));
  const void* fns[4] = {(const void*)k_prep, (const void*)k_post, (const void*)kf_prep, (const void*)kf_post};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rtu
