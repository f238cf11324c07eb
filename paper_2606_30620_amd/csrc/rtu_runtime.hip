// Host runtime of the C ABI declared in include/rtu.h: plans, their device
// memory, observation upload and the launch sequence of one evaluation.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "rtu_internal.h"

using namespace rtu;

// HIP events around the stages of up to max_calls evaluations
struct Prof {
  bool on = false;
  uint32_t mask = 0;
  int max_calls = 0, calls = 0, cur = -1;
  std::vector<hipEvent_t> ev;      // [max_calls][RTU_N_STAGES][2]
  std::vector<uint8_t> used;       // [max_calls][RTU_N_STAGES]
};

struct rtu_plan_s {
  rtu_geometry g;
  int max_batch = 0;
  int device = 0;
  SysDev h;                       // geometry, observation and workspace pointers
  char* pool = nullptr;           // workspace allocation (independent of M)
  char* obs_pool = nullptr;       // observation + M-dependent buffers, sized for M = N^2
  char* stage = nullptr;          // pinned host image of the observation region (one copy per call)
  size_t obs_bytes = 0;
  hipEvent_t stage_done = nullptr;   // the last copy out of `stage` has finished
  bool stage_pending = false;
  int M = -1;
  SysDev last;                    // descriptor of the last evaluation (debug fetch)
  bool have_last = false;
  Prof prof;
  std::vector<float> inv_var;     // host copy of 1/sigma^2 (ELBO constant)
  std::vector<int> mask_idx;      // host copy of the masked pixels (ray weights)
  // weighted RTU grid: device [M] weights, [K] positions, [K] fractions, sort
  // scratch; its pinned staging copy and the event of its last upload
  char* wdev = nullptr;
  size_t wdev_bytes = 0;
  char* wstage = nullptr;
  size_t wstage_bytes = 0;
  hipEvent_t wdone = nullptr;
  bool wpending = false;
};

struct rtu_fit_s {
  rtu_plan plan = nullptr;
  FitDev F;
  char* pool = nullptr;
  int max_steps = 0, steps = 0;
  bool drawn = false;             // the next step's samples are drawn (by the last Adam update)
  int n_sub = 0;
  // the fit runs the shared-launch kernels of the serving fleet on a one-fit
  // table, so a fit alone and a fit in a fleet execute the same code
  DeviceTables tables;
  FleetLaunch L{};
};

namespace rtu {

std::mutex g_const_mu;
std::vector<int> g_const_done;    // devices whose constant tables are uploaded

int ensure_constants(int device) {
  std::lock_guard<std::mutex> lk(g_const_mu);
  for (int d : g_const_done)
    if (d == device) return RTU_OK;
  if (upload_constants() != hipSuccess) return RTU_EHIP;
  g_const_done.push_back(device);
  return RTU_OK;
}

bool valid_geometry(const rtu_geometry* g) {
  if (!g) return false;
  const int n = g->n_src;
  if (g->n_img < 8 || g->n_img > 1024) return false;
  if (g->supersample < 1 || g->supersample > 8) return false;
  if (n < 8 || n > 256 || (n & (n - 1))) return false;
  if (g->psf_size < 1 || g->psf_size > 63 || !(g->psf_size & 1)) return false;
  if (g->n_sub_max < 0 || g->n_sub_max > RTU_MAX_SUB) return false;
  if (g->n_gauss < 0 || g->n_gauss > RTU_MAX_GAUSS) return false;
  if (g->k_nodes != RTU_K_NODES) return false;
  if (!(g->pixel_scale > 0.f) || !(g->tnfw_tau >= 0.f) || (g->flags & ~(RTU_GEOM_RADIX_SELECT | RTU_GEOM_UNIFORM | RTU_GEOM_EPL)) != 0) return false;
  return true;
}

struct Carve {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

void fill_geometry(const rtu_geometry* g, SysDev& h) {
  memset(&h, 0, sizeof(h));
  h.round0 = 0;
  h.nsteps = 0x7fffffff;
  h.n_img = g->n_img;
  h.ss = g->supersample;
  h.n_src = g->n_src;
  int l = 0;
  while ((1 << l) < g->n_src) ++l;
  h.log2_src = l;
  h.psf_k = g->psf_size;
  h.n_sub_max = g->n_sub_max;
  h.n_gauss = g->n_gauss;
  h.light_off = ((g->flags & RTU_GEOM_EPL) ? RTU_N_LENS_BASE_EPL : RTU_N_LENS_BASE) + RTU_N_PER_SUB * g->n_sub_max;
  h.n_lens = h.light_off + RTU_N_PER_GAUSS * g->n_gauss;
  h.pix = g->pixel_scale;
  h.tau = g->tnfw_tau;
  h.inv_ss2 = 1.f / (float)(g->supersample * g->supersample);
  h.sel_radix = (g->flags & RTU_GEOM_RADIX_SELECT) ? 1 : 0;
  h.uniform = (g->flags & RTU_GEOM_UNIFORM) ? 1 : 0;
  h.epl = (g->flags & RTU_GEOM_EPL) ? 1 : 0;
  h.lens_base = h.epl ? RTU_N_LENS_BASE_EPL : RTU_N_LENS_BASE;
  h.ray_tx = (g->n_img + RAY_TILE - 1) / RAY_TILE;
  h.ray_tiles = h.ray_tx * h.ray_tx;
  h.adj_wcap = adj_window_cap(h);
  h.psf_tx = (g->n_img + PSF_TW - 1) / PSF_TW;
  h.psf_tiles = h.psf_tx * ((g->n_img + PSF_TH - 1) / PSF_TH);
}

// workspace independent of the mask
size_t carve_workspace(SysDev& h, int B, char* base) {
  Carve c{base};
  const size_t n2 = (size_t)h.n_src * h.n_src, N2 = (size_t)h.n_img * h.n_img;
  h.src = c.take<float>(B * n2);
  h.srcp = c.take<float>((size_t)B * (h.n_src + 2) * (h.n_src + 2));
  h.fld = c.take<float>(B * n2);
  h.F = c.take<float2>(B * n2);
  h.tmp = c.take<float2>(B * n2);
  h.gpp = c.take<double>((size_t)B * (h.n_src / GP_LINES + 1) * 4);
  h.knots = c.take<float>((size_t)B * 4 * K);
  h.ktab = c.take<KnotTab>((size_t)B);
  h.sie = c.take<Sie>((size_t)B);
  h.kdbg = c.take<float>((size_t)B * 4 * K);
  h.sel = c.take<int>((size_t)B * 4 * K);
  h.stdv = c.take<double>((size_t)B * 4);
  h.dp = c.take<float>((size_t)B * 2 * K);
  h.u = c.take<float>(B * N2);
  h.r = c.take<float>(B * N2);
  h.ubar = c.take<float>(B * N2);
  h.sbar = c.take<double>(B * n2);
  h.kbar = c.take<double>((size_t)B * h.ray_tiles * 4 * K);
  h.tbox = c.take<int4>((size_t)B * h.ray_tiles * (RAY_THREADS / 64));
  h.lpart = c.take<double>((size_t)B * h.ray_tiles * (RAY_THREADS / 64) * (h.n_lens + 2));
  h.c2part = c.take<double>((size_t)B * h.psf_tiles * 2);
  h.st = c.take<uint32_t>((size_t)B * ST_WORDS);
  return c.off + 256;
}

// observation and mask-dependent buffers
size_t carve_observation(SysDev& h, int B, int M, char* base) {
  Carve c{base};
  const size_t N2 = (size_t)h.n_img * h.n_img, kw = (size_t)h.psf_k * psf_ws(h.psf_k);
  h.image = c.take<float>(N2);
  h.inv_var = c.take<float>(N2);
  h.psf_flip = c.take<float>(kw);
  h.psf = c.take<float>(kw);
  h.psf_sep = c.take<float>((size_t)4 * h.psf_k);
  h.mask = c.take<uint8_t>(N2);
  h.mask_idx = c.take<int>(M > 0 ? M : 1);
  h.mask_xy = c.take<float2>(M > 0 ? M : 1);
  h.rank_j = c.take<int>(K);
  h.rank_t = c.take<double>(K);
  h.tsel = c.take<int>(4 * K + 1);
  h.zbuf = c.take<float>((size_t)B * 2 * (M > 0 ? M : 1));
  h.mr_nchunk = mr_chunks(M);
  h.mrp = c.take<MRayPart>((size_t)B * (h.mr_nchunk > 0 ? h.mr_nchunk : 1));
  return c.off + 256;
}

// Host side of an observation: masked pixel list, quantile ranks
// h_k = (M-1) u_k in FP64, inverse variances and the PSF weight rows of both
// correlations (the flipped PSF forward, the PSF as given for the adjoint),
// zero-padded as the matrix-core PSF kernel reads them.
void prepare_observation(const rtu_geometry* g, const float* noise_sigma, const float* psf,
                         const uint8_t* arc_mask, ObsHost& o) {
  const int N = g->n_img, KP = g->psf_size;
  const size_t N2 = (size_t)N * N;
  o.idx.clear();
  o.xy.clear();
  for (size_t q = 0; q < N2; ++q)
    if (arc_mask[q]) {
      o.idx.push_back((int)q);
      o.xy.push_back(pixel_centre((int)q, N, g->pixel_scale));
    }
  const int M = (int)o.idx.size();
  for (int k = 0; k < K; ++k) {
    const double u = 0.5 * (1.0 - cos((2.0 * (k + 1) - 1.0) * M_PI / (2.0 * K)));
    const double hh = (double)(M > 0 ? M - 1 : 0) * u;
    const double fl = floor(hh);
    o.rank_j[k] = (int)fl;
    o.rank_t[k] = hh - fl;
  }
  target_list(o.rank_j, M, o.tsel);
  o.inv_var.resize(N2);
  for (size_t q = 0; q < N2; ++q) o.inv_var[q] = 1.f / (noise_sigma[q] * noise_sigma[q]);
  const int WS = psf_ws(KP);
  o.wfwd.assign((size_t)KP * WS, 0.f);
  o.wadj.assign((size_t)KP * WS, 0.f);
  for (int a = 0; a < KP; ++a)
    for (int b = 0; b < KP; ++b) {
      o.wfwd[(size_t)a * WS + b + 15] = psf[(size_t)(KP - 1 - a) * KP + (KP - 1 - b)];
      o.wadj[(size_t)a * WS + b + 15] = psf[(size_t)a * KP + b];
    }
  // Rank one (a Gaussian PSF is): W[a][c] = u[a] v[c] with u the column and v
  // the row through the largest weight, accepted when every weight is
  // reproduced to a few FP32 ulps of the largest one.
  o.wsep.assign((size_t)4 * KP, 0.f);
  o.rank1 = false;
  int ar = 0, ac = 0;
  double wmax = 0.0;
  for (int a = 0; a < KP; ++a)
    for (int b = 0; b < KP; ++b)
      if (std::fabs((double)psf[(size_t)a * KP + b]) > wmax) {
        wmax = std::fabs((double)psf[(size_t)a * KP + b]);
        ar = a;
        ac = b;
      }
  if (wmax > 0.0) {
    std::vector<float> u(KP), v(KP);
    const double piv = psf[(size_t)ar * KP + ac];
    for (int a = 0; a < KP; ++a) u[a] = psf[(size_t)a * KP + ac];
    for (int b = 0; b < KP; ++b) v[b] = (float)((double)psf[(size_t)ar * KP + b] / piv);
    double err = 0.0;
    for (int a = 0; a < KP; ++a)
      for (int b = 0; b < KP; ++b)
        err = std::max(err, std::fabs((double)psf[(size_t)a * KP + b] - (double)u[a] * (double)v[b]));
    o.rank1 = err <= 4e-7 * wmax;
    for (int a = 0; a < KP; ++a) {
      o.wsep[a] = u[KP - 1 - a];                 // forward: the flipped PSF
      o.wsep[KP + a] = v[KP - 1 - a];
      o.wsep[2 * KP + a] = u[a];                 // adjoint: the PSF as given
      o.wsep[3 * KP + a] = v[a];
    }
  }
}

hipError_t upload_observation(const SysDev& h, const float* image, const float* psf, const uint8_t* arc_mask,
                              const ObsHost& o, hipStream_t s) {
  const size_t N2 = (size_t)h.n_img * h.n_img, kw = (size_t)h.psf_k * psf_ws(h.psf_k);
  hipError_t e = hipSuccess;
  auto cp = [&](const void* dst, const void* src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpyAsync(const_cast<void*>(dst), src, n, hipMemcpyHostToDevice, s);
  };
  cp(h.image, image, N2 * 4);
  cp(h.inv_var, o.inv_var.data(), N2 * 4);
  cp(h.psf_flip, o.wfwd.data(), kw * 4);
  cp(h.psf, o.wadj.data(), kw * 4);
  cp(h.psf_sep, o.wsep.data(), o.wsep.size() * 4);
  cp(h.mask, arc_mask, N2);
  cp(h.mask_idx, o.idx.data(), o.idx.size() * 4);
  cp(h.mask_xy, o.xy.data(), o.xy.size() * sizeof(float2));
  cp(h.rank_j, o.rank_j, sizeof(o.rank_j));
  cp(h.rank_t, o.rank_t, sizeof(o.rank_t));
  cp(h.tsel, o.tsel, sizeof(o.tsel));
  return e;
}

// Fit state of S samples: guide, Adam moments, sample and gradient buffers.
size_t carve_fit(FitDev& F, int S, int max_steps, char* base) {
  Carve cv{base};
  F.mu = cv.take<float>(F.dim); F.rho = cv.take<float>(F.dim);
  F.m_mu = cv.take<float>(F.dim); F.v_mu = cv.take<float>(F.dim);
  F.m_rho = cv.take<float>(F.dim); F.v_rho = cv.take<float>(F.dim);
  F.z_lens = cv.take<float>((size_t)S * F.n_lens); F.z_ps = cv.take<float>((size_t)S * 4);
  F.z_lat = cv.take<float>((size_t)S * F.n_src2);
  F.g_lens = cv.take<float>((size_t)S * F.n_lens); F.g_ps = cv.take<float>((size_t)S * 4);
  F.g_lat = cv.take<float>((size_t)S * F.n_src2);
  F.eps_s = cv.take<float>((size_t)S * F.dim);
  F.loss = cv.take<double>(S); F.chi2m = cv.take<double>(S);
  F.status = cv.take<uint32_t>(S); F.n_sub = cv.take<int>(S);
  F.trace = cv.take<double>(max_steps);
  F.status_acc = cv.take<uint32_t>(1);
  F.rho_part = cv.take<double>(2 * (((size_t)F.dim + ADAM_P - 1) / ADAM_P));
  return cv.off + 256;
}

// ELBO constant: -sum_p ln(sigma_p sqrt(2 pi)) - (n^2/2) ln 2 pi + (dim/2)(1 + ln 2 pi)
double elbo_constant(const std::vector<float>& inv_var, int n_src2, int dim) {
  double c = 0.0;
  for (float v : inv_var) c += 0.5 * log((double)v) - 0.5 * log(2.0 * M_PI);
  return c - 0.5 * n_src2 * log(2.0 * M_PI) + 0.5 * dim * (1.0 + log(2.0 * M_PI));
}

// Initial fit state on the device: mu, rho, zero moments, n_sub per sample.
hipError_t init_fit_state(const FitDev& F, const float* mu0, const float* rho0, int n_sub, hipStream_t s) {
  std::vector<int> ns(F.S, n_sub);
  hipError_t e = hipMemcpyAsync(F.mu, mu0, (size_t)F.dim * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(F.rho, rho0, (size_t)F.dim * 4, hipMemcpyHostToDevice, s);
  float* z[4] = {F.m_mu, F.v_mu, F.m_rho, F.v_rho};
  for (int k = 0; k < 4 && e == hipSuccess; ++k) e = hipMemsetAsync(z[k], 0, (size_t)F.dim * 4, s);
  if (e == hipSuccess && F.status_acc) e = hipMemsetAsync(F.status_acc, 0, 4, s);
  if (e == hipSuccess) e = hipMemcpyAsync(F.n_sub, ns.data(), (size_t)F.S * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host vector above must outlive the copy
  return e;
}

}  // namespace rtu

// The allocation-free entry point keeps every intermediate in this array.
// Each device holds its own copy at its own address, found once per device
// with hipGetSymbolAddress; host code uses only that address, never the
// array's name.
static __device__ __align__(256) char scratch[RTU_NOALLOC_MAX_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<std::pair<int, char*>> g_scratch;   // (device, address of its copy)

// Set-up on the current device, once: the constant tables and the address of
// its copy of the array.
int scratch_base(int device, char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  for (const auto& d : g_scratch)
    if (d.first == device) {
      *out = d.second;
      return RTU_OK;
    }
  const int rc = ensure_constants(device);
  if (rc) return rc;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RTU_EHIP;
  g_scratch.emplace_back(device, static_cast<char*>(ptr));
  *out = static_cast<char*>(ptr);
  return RTU_OK;
}

void prof_call_begin(rtu_plan p) {
  Prof& P = p->prof;
  P.cur = (P.on && P.calls < P.max_calls) ? P.calls++ : -1;
}
void prof_stage(rtu_plan p, int stage, bool end, hipStream_t s) {
  Prof& P = p->prof;
  if (P.cur < 0 || !(P.mask & (1u << stage))) return;
  const size_t q = (size_t)P.cur * RTU_N_STAGES + stage;
  (void)hipEventRecord(P.ev[q * 2 + (end ? 1 : 0)], s);
  if (end) P.used[q] = 1;
}

// The launch sequence of one evaluation of `batch` samples.
int run_eval(rtu_plan p, const SysDev& h, int batch, hipStream_t s) {
  prof_stage(p, RTU_STAGE_PREP, false, s);
  if (launch_prep(h, batch, s) != hipSuccess) return RTU_EHIP;
  prof_stage(p, RTU_STAGE_PREP, true, s);
  prof_stage(p, RTU_STAGE_RAYS_FWD, false, s);
  if (launch_rays_fwd(h, batch, s) != hipSuccess) return RTU_EHIP;
  prof_stage(p, RTU_STAGE_RAYS_FWD, true, s);
  prof_stage(p, RTU_STAGE_PSF_FWD, false, s);
  if (launch_psf(h, batch, false, s) != hipSuccess) return RTU_EHIP;
  prof_stage(p, RTU_STAGE_PSF_FWD, true, s);
  if (h.want_grad) {
    prof_stage(p, RTU_STAGE_PSF_ADJ, false, s);
    if (launch_psf(h, batch, true, s) != hipSuccess) return RTU_EHIP;
    prof_stage(p, RTU_STAGE_PSF_ADJ, true, s);
    prof_stage(p, RTU_STAGE_RAYS_ADJ, false, s);
    if (launch_rays_adj(h, batch, s) != hipSuccess) return RTU_EHIP;
    prof_stage(p, RTU_STAGE_RAYS_ADJ, true, s);
  }
  prof_stage(p, RTU_STAGE_POST, false, s);
  if (launch_post(h, batch, s) != hipSuccess) return RTU_EHIP;
  prof_stage(p, RTU_STAGE_POST, true, s);
  p->last = h;
  p->have_last = true;
  return RTU_OK;
}

}  // namespace

extern "C" {

int32_t rtu_n_lens(const rtu_geometry* g) {
  return g ? ((g->flags & RTU_GEOM_EPL) ? RTU_N_LENS_BASE_EPL : RTU_N_LENS_BASE) + RTU_N_PER_SUB * g->n_sub_max +
                 RTU_N_PER_GAUSS * g->n_gauss
           : 0;
}

size_t rtu_workspace_bytes(const rtu_geometry* g, int32_t max_batch) {
  if (!valid_geometry(g) || max_batch < 1) return 0;
  SysDev h;
  fill_geometry(g, h);
  return carve_workspace(h, max_batch, nullptr) +
         carve_observation(h, max_batch, g->n_img * g->n_img, nullptr);
}

int rtu_plan_create(const rtu_geometry* g, int32_t max_batch, int32_t device, rtu_plan* out) {
  if (!out || !valid_geometry(g) || max_batch < 1) return RTU_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return RTU_EINVAL;
  int rc = ensure_constants(device);
  if (rc) return rc;
  rtu_plan p = new rtu_plan_s();
  p->g = *g;
  p->max_batch = max_batch;
  p->device = device;
  fill_geometry(g, p->h);
  const size_t bytes = carve_workspace(p->h, max_batch, nullptr);
  // the observation region for any mask (M <= N^2), so that a new observation
  // never reallocates
  SysDev tmp = p->h;
  p->obs_bytes = carve_observation(tmp, max_batch, g->n_img * g->n_img, nullptr);
  if (hipMalloc(&p->pool, bytes) != hipSuccess || hipMalloc(&p->obs_pool, p->obs_bytes) != hipSuccess ||
      hipHostMalloc(&p->stage, p->obs_bytes, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&p->stage_done, hipEventDisableTiming) != hipSuccess) {
    if (p->pool) (void)hipFree(p->pool);
    if (p->obs_pool) (void)hipFree(p->obs_pool);
    if (p->stage) (void)hipHostFree(p->stage);
    if (p->stage_done) (void)hipEventDestroy(p->stage_done);
    delete p;
    return RTU_ENOMEM;
  }
  carve_workspace(p->h, max_batch, p->pool);
  *out = p;
  return RTU_OK;
}

int rtu_plan_destroy(rtu_plan p) {
  if (!p) return RTU_EINVAL;
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  if (p->pool) (void)hipFree(p->pool);
  if (p->obs_pool) (void)hipFree(p->obs_pool);
  if (p->stage) (void)hipHostFree(p->stage);
  if (p->stage_done) (void)hipEventDestroy(p->stage_done);
  if (p->wdev) (void)hipFree(p->wdev);
  if (p->wstage) (void)hipHostFree(p->wstage);
  if (p->wdone) (void)hipEventDestroy(p->wdone);
  for (hipEvent_t e : p->prof.ev) (void)hipEventDestroy(e);
  delete p;
  return RTU_OK;
}

int rtu_set_observation(rtu_plan p, const float* image, const float* noise_sigma, const float* psf,
                        const uint8_t* arc_mask, void* stream) {
  if (!p || !image || !noise_sigma || !psf || !arc_mask) return RTU_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return RTU_EHIP;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ObsHost o;
  prepare_observation(&p->g, noise_sigma, psf, arc_mask, o);
  const int M = (int)o.idx.size();
  // the pinned staging buffer still feeds the previous call's copy until its
  // event has passed (that copy only: no other work is waited for)
  if (p->stage_pending && hipEventSynchronize(p->stage_done) != hipSuccess) return RTU_EHIP;
  p->stage_pending = false;
  // the observation region laid out in the staging buffer exactly as on the
  // device (same offsets), filled, then sent in one asynchronous copy
  SysDev hs = p->h, h = p->h;
  carve_observation(hs, p->max_batch, M, p->stage);
  carve_observation(h, p->max_batch, M, p->obs_pool);
  const size_t N2 = (size_t)h.n_img * h.n_img, kw = (size_t)h.psf_k * psf_ws(h.psf_k);
  memcpy(const_cast<float*>(hs.image), image, N2 * 4);
  memcpy(const_cast<float*>(hs.inv_var), o.inv_var.data(), N2 * 4);
  memcpy(const_cast<float*>(hs.psf_flip), o.wfwd.data(), kw * 4);
  memcpy(const_cast<float*>(hs.psf), o.wadj.data(), kw * 4);
  memcpy(const_cast<float*>(hs.psf_sep), o.wsep.data(), o.wsep.size() * 4);
  memcpy(const_cast<uint8_t*>(hs.mask), arc_mask, N2);
  if (M) memcpy(const_cast<int*>(hs.mask_idx), o.idx.data(), (size_t)M * 4);
  if (M) memcpy(const_cast<float2*>(hs.mask_xy), o.xy.data(), (size_t)M * sizeof(float2));
  memcpy(const_cast<int*>(hs.rank_j), o.rank_j, sizeof(o.rank_j));
  memcpy(const_cast<double*>(hs.rank_t), o.rank_t, sizeof(o.rank_t));
  memcpy(const_cast<int*>(hs.tsel), o.tsel, sizeof(o.tsel));
  const size_t bytes = (size_t)(reinterpret_cast<const char*>(h.zbuf) - p->obs_pool);
  if (hipMemcpyAsync(p->obs_pool, p->stage, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return RTU_EHIP;
  if (hipEventRecord(p->stage_done, s) != hipSuccess) return RTU_EHIP;
  p->stage_pending = true;
  h.M = M;
  h.psf_rank1 = o.rank1 ? 1 : 0;
  // a new mask: the ray weights, if any, must be given again
  h.ray_w = nullptr; h.wr0 = nullptr; h.wt = nullptr; h.wsort = nullptr; h.wsum = 0.0;
  p->h = h;
  p->M = M;
  p->inv_var = o.inv_var;
  p->mask_idx = o.idx;
  return RTU_OK;
}

int rtu_set_ray_weights(rtu_plan p, const float* weights, void* stream) {
  if (!p) return RTU_EINVAL;
  if (p->M < 0) return RTU_ESTATE;
  if (hipSetDevice(p->device) != hipSuccess) return RTU_EHIP;
  SysDev& h = p->h;
  if (!weights) {
    h.ray_w = nullptr; h.wr0 = nullptr; h.wt = nullptr; h.wsort = nullptr; h.wsum = 0.0;
    return RTU_OK;
  }
  const int M = p->M;
  double W = 0.0;
  for (int m = 0; m < M; ++m) {
    const float w = weights[p->mask_idx[m]];
    if (!(w >= 0.f) || !std::isfinite(w)) return RTU_EINVAL;
    W += (double)w;
  }
  if (!(W >= 1.0)) return RTU_EINVAL;
  // device layout: weights [M] (float), positions [K], fractions [K] (double),
  // then the sort scratch [max_batch][2][2][M] (uint2)
  const size_t off_r = (((size_t)M * 4 + 15) & ~(size_t)15), off_s = off_r + 2 * K * sizeof(double);
  const size_t host_bytes = off_s, bytes = off_s + (size_t)p->max_batch * 4 * M * sizeof(uint2);
  if (p->wpending && hipEventSynchronize(p->wdone) != hipSuccess) return RTU_EHIP;
  p->wpending = false;
  if (bytes > p->wdev_bytes) {
    // the previous array may still be read by queued work
    if (p->wdev && (hipDeviceSynchronize() != hipSuccess || hipFree(p->wdev) != hipSuccess)) return RTU_EHIP;
    p->wdev = nullptr;
    p->wdev_bytes = 0;
    h.ray_w = nullptr;
    if (hipMalloc(&p->wdev, bytes) != hipSuccess) return RTU_ENOMEM;
    p->wdev_bytes = bytes;
  }
  if (host_bytes > p->wstage_bytes) {
    if (p->wstage) (void)hipHostFree(p->wstage);
    p->wstage = nullptr;
    p->wstage_bytes = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&p->wstage), host_bytes, hipHostMallocDefault) != hipSuccess)
      return RTU_ENOMEM;
    p->wstage_bytes = host_bytes;
  }
  if (!p->wdone && hipEventCreateWithFlags(&p->wdone, hipEventDisableTiming) != hipSuccess) return RTU_EHIP;
  float* hw = reinterpret_cast<float*>(p->wstage);
  double* hr = reinterpret_cast<double*>(p->wstage + off_r);
  for (int m = 0; m < M; ++m) hw[m] = weights[p->mask_idx[m]];
  for (int k = 0; k < K; ++k) {
    const double u = 0.5 * (1.0 - cos((2.0 * (k + 1) - 1.0) * M_PI / (2.0 * K)));
    const double hh = (W - 1.0) * u, fl = floor(hh);
    hr[k] = fl;
    hr[K + k] = hh - fl;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (hipMemcpyAsync(p->wdev, p->wstage, host_bytes, hipMemcpyHostToDevice, s) != hipSuccess) return RTU_EHIP;
  if (hipEventRecord(p->wdone, s) != hipSuccess) return RTU_EHIP;
  p->wpending = true;
  h.ray_w = reinterpret_cast<const float*>(p->wdev);
  h.wr0 = reinterpret_cast<const double*>(p->wdev + off_r);
  h.wt = h.wr0 + K;
  h.wsort = reinterpret_cast<uint2*>(p->wdev + off_s);
  h.wsum = W;
  return RTU_OK;
}

int32_t rtu_masked_count(rtu_plan p) { return p ? p->M : -1; }

int rtu_loss_grad_noalloc(const rtu_geometry* g, int32_t batch, const float* image, const float* noise_sigma,
                          const float* psf, const uint8_t* arc_mask, const float* lens_params,
                          const int32_t* n_sub, const float* ps_params, const float* latent, double* loss,
                          double* chi2_mask, float* grad_lens, float* grad_ps, float* grad_latent,
                          float* model_image, uint32_t* status, void* stream) {
  if (!valid_geometry(g) || batch < 1) return RTU_EINVAL;
  if (!image || !noise_sigma || !psf || !arc_mask || !lens_params || !ps_params || !latent || !loss || !status)
    return RTU_EINVAL;
  if (reinterpret_cast<uintptr_t>(latent) % 16) return RTU_EINVAL;   // read four floats at a time
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return RTU_EHIP;
  SysDev h;
  fill_geometry(g, h);
  // layout in the static array: workspace, observation tables (room for any
  // mask), the observation's M and rank-one flag
  const size_t ws = carve_workspace(h, batch, nullptr);
  const size_t ob = carve_observation(h, batch, g->n_img * g->n_img, nullptr);
  if (ws + ob + 256 > RTU_NOALLOC_MAX_BYTES) return RTU_ETOOBIG;
  char* base = nullptr;
  const int rc = scratch_base(device, &base);
  if (rc) return rc;
  carve_workspace(h, batch, base);
  carve_observation(h, batch, g->n_img * g->n_img, base + ws);
  h.mr_nchunk = 0;   // M is known on the device only: the selection shoots the rays
  int* dyn = reinterpret_cast<int*>(base + ws + ob);
  // the kernels read the image and the mask where the caller keeps them
  h.image = image;
  h.mask = arc_mask;
  h.obs_dyn = dyn;
  h.batch = batch;
  h.lens = lens_params;
  h.n_sub = n_sub;
  h.ps = ps_params;
  h.latent = latent;
  h.loss = loss;
  h.chi2m = chi2_mask;
  h.g_lens = grad_lens;
  h.g_ps = grad_ps;
  h.g_lat = grad_latent;
  h.model = model_image;
  h.status = status;
  h.want_grad = (grad_lens || grad_ps || grad_latent) ? 1 : 0;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // every scratch value the evaluation reads is written earlier in this call:
  // the observation tables here, the rest by the stages (prep zeroes the
  // source adjoint and the status words), so nothing is cleared
  if (launch_observe(h, noise_sigma, psf, dyn, s) != hipSuccess) return RTU_EHIP;
  if (launch_prep(h, batch, s) != hipSuccess) return RTU_EHIP;
  if (launch_rays_fwd(h, batch, s) != hipSuccess) return RTU_EHIP;
  if (launch_psf(h, batch, false, s) != hipSuccess) return RTU_EHIP;
  if (h.want_grad) {
    if (launch_psf(h, batch, true, s) != hipSuccess) return RTU_EHIP;
    if (launch_rays_adj(h, batch, s) != hipSuccess) return RTU_EHIP;
  }
  if (launch_post(h, batch, s) != hipSuccess) return RTU_EHIP;
  return RTU_OK;
}

int rtu_loss_grad(rtu_plan p, int32_t batch, const float* lens_params, const int32_t* n_sub,
                  const float* ps_params, const float* latent, double* loss, double* chi2_mask,
                  float* grad_lens, float* grad_ps, float* grad_latent, float* model_image,
                  uint32_t* status, void* stream) {
  if (!p) return RTU_EINVAL;
  if (p->M < 0) return RTU_ESTATE;
  if (batch < 1) return RTU_EINVAL;
  if (batch > p->max_batch) return RTU_EBATCH;
  if (!lens_params || !ps_params || !latent || !loss || !status) return RTU_EINVAL;
  if (reinterpret_cast<uintptr_t>(latent) % 16) return RTU_EINVAL;   // read four floats at a time
  if (hipSetDevice(p->device) != hipSuccess) return RTU_EHIP;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  SysDev h = p->h;
  h.batch = batch;
  h.lens = lens_params;
  h.n_sub = n_sub;
  h.ps = ps_params;
  h.latent = latent;
  h.loss = loss;
  h.chi2m = chi2_mask;
  h.g_lens = grad_lens;
  h.g_ps = grad_ps;
  h.g_lat = grad_latent;
  h.model = model_image;
  h.status = status;
  h.want_grad = (grad_lens || grad_ps || grad_latent) ? 1 : 0;
  prof_call_begin(p);
  return run_eval(p, h, batch, s);
}

int rtu_debug_fetch(rtu_plan p, int32_t what, int32_t sample, void* host_dst, size_t bytes, void* stream) {
  if (!p || !host_dst || !p->have_last || sample < 0 || sample >= p->last.batch) return RTU_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return RTU_EHIP;
  const SysDev& h = p->last;
  const void* src = nullptr;
  size_t need = 0;
  const size_t n2 = (size_t)h.n_src * h.n_src, N2 = (size_t)h.n_img * h.n_img;
  switch (what) {
    case RTU_DBG_KNOTS: src = h.kdbg + (size_t)sample * 4 * K; need = 4 * K * sizeof(float); break;
    case RTU_DBG_SELECT: src = h.sel + (size_t)sample * 4 * K; need = 4 * K * sizeof(int); break;
    case RTU_DBG_STD: src = h.stdv + (size_t)sample * 4; need = 3 * sizeof(double); break;
    case RTU_DBG_SOURCE: src = h.src + (size_t)sample * n2; need = n2 * sizeof(float); break;
    case RTU_DBG_PREPSF: src = h.u + (size_t)sample * N2; need = N2 * sizeof(float); break;
    case RTU_DBG_ONGRID: need = sizeof(double); break;
    default: return RTU_EINVAL;
  }
  if (bytes < need) return RTU_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess) return RTU_EHIP;
  if (what == RTU_DBG_ONGRID) {
    if (!h.want_grad) return RTU_ESTATE;
    // the last column of the sample's per-wave lens-gradient rows
    const size_t ld = (size_t)h.n_lens + 2, rows = (size_t)h.ray_tiles * (RAY_THREADS / 64);
    std::vector<double> v(rows * ld);
    if (hipMemcpy(v.data(), h.lpart + (size_t)sample * rows * ld, v.size() * sizeof(double),
                  hipMemcpyDeviceToHost) != hipSuccess)
      return RTU_EHIP;
    double n = 0.0;
    for (size_t r = 0; r < rows; ++r) n += v[r * ld + ld - 1];
    *static_cast<double*>(host_dst) = n;
    return RTU_OK;
  }
  if (hipMemcpy(host_dst, src, need, hipMemcpyDeviceToHost) != hipSuccess) return RTU_EHIP;
  return RTU_OK;
}

int rtu_profile_begin(rtu_plan p, int32_t max_calls, uint32_t stage_mask) {
  if (!p || max_calls < 1) return RTU_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return RTU_EHIP;
  Prof& P = p->prof;
  for (hipEvent_t e : P.ev) (void)hipEventDestroy(e);
  P.ev.assign((size_t)max_calls * RTU_N_STAGES * 2, nullptr);
  P.used.assign((size_t)max_calls * RTU_N_STAGES, 0);
  for (auto& e : P.ev)
    if (hipEventCreate(&e) != hipSuccess) return RTU_EHIP;
  P.on = true;
  P.mask = stage_mask ? stage_mask : (1u << RTU_N_STAGES) - 1u;
  P.max_calls = max_calls;
  P.calls = 0;
  P.cur = -1;
  return RTU_OK;
}

int rtu_profile_end(rtu_plan p, double* stage_ms, int32_t* launches) {
  if (!p || !stage_ms) return RTU_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return RTU_EHIP;
  Prof& P = p->prof;
  for (int k = 0; k < RTU_N_STAGES; ++k) {
    stage_ms[k] = 0.0;
    if (launches) launches[k] = 0;
  }
  for (int c = 0; c < P.calls; ++c)
    for (int k = 0; k < RTU_N_STAGES; ++k) {
      const size_t q = (size_t)c * RTU_N_STAGES + k;
      if (!P.used[q]) continue;
      if (hipEventSynchronize(P.ev[q * 2 + 1]) != hipSuccess) return RTU_EHIP;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, P.ev[q * 2], P.ev[q * 2 + 1]) != hipSuccess) return RTU_EHIP;
      stage_ms[k] += ms;
      if (launches) launches[k] += 1;
    }
  for (hipEvent_t e : P.ev) (void)hipEventDestroy(e);
  P.ev.clear();
  P.used.clear();
  P.on = false;
  P.calls = 0;
  P.cur = -1;
  return RTU_OK;
}

int rtu_fit_create(rtu_plan p, int32_t samples, const float* mu0, const float* rho0, float lr,
                   uint64_t seed, int32_t max_steps, int32_t n_sub, const uint32_t* log_mask, rtu_fit* out) {
  if (!p || !out || !mu0 || !rho0 || samples < 1 || max_steps < 1) return RTU_EINVAL;
  if (samples > p->max_batch) return RTU_EBATCH;
  if (p->M < 0) return RTU_ESTATE;
  if (n_sub < 0 || n_sub > p->g.n_sub_max) return RTU_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return RTU_EHIP;
  rtu_fit f = new rtu_fit_s();
  f->plan = p;
  f->max_steps = max_steps;
  f->n_sub = n_sub;
  FitDev& F = f->F;
  memset(&F, 0, sizeof(F));
  const int S = samples, nl = p->h.n_lens, n2 = p->h.n_src * p->h.n_src;
  F.S = S;
  F.n_lens = nl;
  F.n_src2 = n2;
  F.dim = nl + 4 + n2;
  F.lr = lr;
  F.seed_lo = (uint32_t)seed;
  F.seed_hi = (uint32_t)(seed >> 32);
  for (int w = 0; w < RTU_LOG_MASK_WORDS; ++w) F.log_mask[w] = log_mask ? log_mask[w] : 0u;
  F.round0 = 0;
  F.nsteps = max_steps;
  F.elbo_const = elbo_constant(p->inv_var, n2, F.dim);
  const size_t bytes = carve_fit(F, S, max_steps, nullptr);
  if (hipMalloc(&f->pool, bytes) != hipSuccess) {
    delete f;
    return RTU_ENOMEM;
  }
  carve_fit(F, S, max_steps, f->pool);
  if (init_fit_state(F, mu0, rho0, n_sub, nullptr) != hipSuccess) {
    (void)hipFree(f->pool);
    delete f;
    return RTU_EHIP;
  }
  SysDev h = p->h;
  h.batch = S;
  h.want_grad = 1;
  h.lens = F.z_lens; h.n_sub = F.n_sub; h.ps = F.z_ps; h.latent = F.z_lat;
  h.loss = F.loss; h.chi2m = F.chi2m; h.g_lens = F.g_lens; h.g_ps = F.g_ps; h.g_lat = F.g_lat;
  h.model = nullptr; h.status = F.status;
  h.lds_adj = adj_lds_grid(h) ? 1 : 0;
  h.round0 = 0;
  h.nsteps = max_steps;
  const int rc = f->tables.upload({h}, {F}, f->L);
  if (rc) {
    f->tables.release();
    (void)hipFree(f->pool);
    delete f;
    return rc;
  }
  p->last = h;
  p->have_last = true;
  *out = f;
  return RTU_OK;
}

int rtu_fit_destroy(rtu_fit f) {
  if (!f) return RTU_EINVAL;
  (void)hipSetDevice(f->plan->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(f->pool);
  f->tables.release();
  delete f;
  return RTU_OK;
}

int32_t rtu_fit_dim(rtu_fit f) { return f ? f->F.dim : -1; }

int rtu_fit_step(rtu_fit f, int32_t n_steps, const float* eps, void* stream) {
  if (!f || n_steps < 0) return RTU_EINVAL;
  if (f->steps + n_steps > f->max_steps) return RTU_EINVAL;
  rtu_plan p = f->plan;
  if (p->M < 0) return RTU_ESTATE;
  if (hipSetDevice(p->device) != hipSuccess) return RTU_EHIP;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const FitDev& F = f->F;
  const int order[] = {RTU_STAGE_SAMPLE, RTU_STAGE_PREP, RTU_STAGE_RAYS_FWD, RTU_STAGE_PSF_FWD,
                       RTU_STAGE_PSF_ADJ, RTU_STAGE_RAYS_ADJ, RTU_STAGE_POST, RTU_STAGE_ADAM};
  for (int k = 0; k < n_steps; ++k) {
    const int step = f->steps;
    const float* ek = eps ? eps + (size_t)k * F.S * F.dim : nullptr;
    prof_call_begin(p);
    for (int st : order) {
      if (st == RTU_STAGE_SAMPLE && f->drawn && !ek) continue;
      prof_stage(p, st, false, s);
      if (launch_fleet_stage(f->L, st, step, ek, s) != hipSuccess) return RTU_EHIP;
      prof_stage(p, st, true, s);
    }
    f->drawn = ek == nullptr;      // Philox draws: the Adam update drew the next step's samples
    f->steps++;
  }
  return RTU_OK;
}

int rtu_fit_read(rtu_fit f, float* mu, float* rho, double* elbo, int32_t max_trace, int32_t* n_trace,
                 uint32_t* status, void* stream) {
  if (!f) return RTU_EINVAL;
  if (hipSetDevice(f->plan->device) != hipSuccess) return RTU_EHIP;
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return RTU_EHIP;
  const FitDev& F = f->F;
  hipError_t e = hipSuccess;
  if (mu) e = hipMemcpy(mu, F.mu, (size_t)F.dim * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && rho) e = hipMemcpy(rho, F.rho, (size_t)F.dim * 4, hipMemcpyDeviceToHost);
  const int nt = f->steps < max_trace ? f->steps : max_trace;
  if (e == hipSuccess && elbo && nt > 0) e = hipMemcpy(elbo, F.trace, (size_t)nt * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess && status) e = hipMemcpy(status, F.status_acc, 4, hipMemcpyDeviceToHost);
  if (n_trace) *n_trace = f->steps;
  return e == hipSuccess ? RTU_OK : RTU_EHIP;
}

int rtu_fit_get_state(rtu_fit f, float* state, int32_t* steps, void* stream) {
  if (!f || !state) return RTU_EINVAL;
  if (hipSetDevice(f->plan->device) != hipSuccess) return RTU_EHIP;
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return RTU_EHIP;
  const FitDev& F = f->F;
  float* src[6] = {F.mu, F.rho, F.m_mu, F.v_mu, F.m_rho, F.v_rho};
  for (int k = 0; k < 6; ++k)
    if (hipMemcpy(state + (size_t)k * F.dim, src[k], (size_t)F.dim * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return RTU_EHIP;
  if (steps) *steps = f->steps;
  return RTU_OK;
}

int rtu_fit_set_state(rtu_fit f, const float* state, int32_t steps) {
  if (!f || !state || steps < 0 || steps > f->max_steps) return RTU_EINVAL;
  if (hipSetDevice(f->plan->device) != hipSuccess) return RTU_EHIP;
  const FitDev& F = f->F;
  float* dst[6] = {F.mu, F.rho, F.m_mu, F.v_mu, F.m_rho, F.v_rho};
  if (hipDeviceSynchronize() != hipSuccess) return RTU_EHIP;
  for (int k = 0; k < 6; ++k)
    if (hipMemcpy(dst[k], state + (size_t)k * F.dim, (size_t)F.dim * 4, hipMemcpyHostToDevice) != hipSuccess)
      return RTU_EHIP;
  f->steps = steps;
  f->drawn = false;
  return RTU_OK;
}

int rtu_fit_samples(rtu_fit f, float* z, void* stream) {
  if (!f || !z) return RTU_EINVAL;
  if (hipSetDevice(f->plan->device) != hipSuccess) return RTU_EHIP;
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return RTU_EHIP;
  const FitDev& F = f->F;
  for (int s = 0; s < F.S; ++s) {
    float* row = z + (size_t)s * F.dim;
    if (hipMemcpy(row, F.z_lens + (size_t)s * F.n_lens, (size_t)F.n_lens * 4, hipMemcpyDeviceToHost) ||
        hipMemcpy(row + F.n_lens, F.z_ps + (size_t)s * 4, 16, hipMemcpyDeviceToHost) ||
        hipMemcpy(row + F.n_lens + 4, F.z_lat + (size_t)s * F.n_src2, (size_t)F.n_src2 * 4,
                  hipMemcpyDeviceToHost))
      return RTU_EHIP;
  }
  return RTU_OK;
}

int rtu_fit_last_outputs(rtu_fit f, const double** loss, const uint32_t** status) {
  if (!f) return RTU_EINVAL;
  if (loss) *loss = f->F.loss;
  if (status) *status = f->F.status;
  return RTU_OK;
}

const char* rtu_strerror(int code) {
  switch (code) {
    case RTU_OK: return "ok";
    case RTU_EINVAL: return "invalid argument or geometry";
    case RTU_ENOMEM: return "device memory allocation failed or budget exceeded";
    case RTU_EBATCH: return "batch larger than the plan's max_batch";
    case RTU_EHIP: return "HIP runtime call or kernel launch failed";
    case RTU_ESTATE: return "call out of order (no observation set)";
    case RTU_ENOTFOUND: return "unknown fit id";
    case RTU_ETOOBIG: return "geometry and batch need more than the static scratch array (RTU_NOALLOC_MAX_BYTES)";
    default: return "unknown error";
  }
}

}  // extern "C"
