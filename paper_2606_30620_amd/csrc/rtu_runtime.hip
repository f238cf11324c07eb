// Host runtime of the C ABI declared in include/rtu.h: plans, their device
// memory, observation upload and the launch sequence of one evaluation.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "rtu_internal.h"

using namespace rtu;

struct rtu_plan_s {
  rtu_geometry g;
  int max_batch = 0;
  int device = 0;
  SysDev h;                       // geometry, observation and workspace pointers
  char* pool = nullptr;           // workspace allocation (independent of M)
  char* obs_pool = nullptr;       // observation + M-dependent buffers
  size_t obs_bytes = 0;
  int M = -1;
  SysDev last;                    // descriptor of the last evaluation (debug fetch)
  bool have_last = false;
};

namespace {

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
  if (g->k_nodes != RTU_K_NODES) return false;
  if (!(g->pixel_scale > 0.f) || !(g->tnfw_tau >= 0.f) || g->flags != 0) return false;
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
  h.n_img = g->n_img;
  h.ss = g->supersample;
  h.n_src = g->n_src;
  int l = 0;
  while ((1 << l) < g->n_src) ++l;
  h.log2_src = l;
  h.psf_k = g->psf_size;
  h.n_sub_max = g->n_sub_max;
  h.n_lens = RTU_N_LENS_BASE + RTU_N_PER_SUB * g->n_sub_max;
  h.pix = g->pixel_scale;
  h.tau = g->tnfw_tau;
  h.inv_ss2 = 1.f / (float)(g->supersample * g->supersample);
  h.ray_tx = (g->n_img + RAY_TILE - 1) / RAY_TILE;
  h.ray_tiles = h.ray_tx * h.ray_tx;
  h.psf_tx = (g->n_img + PSF_TW - 1) / PSF_TW;
  h.psf_tiles = h.psf_tx * ((g->n_img + PSF_TH - 1) / PSF_TH);
}

// workspace independent of the mask
size_t carve_workspace(SysDev& h, int B, char* base) {
  Carve c{base};
  const size_t n2 = (size_t)h.n_src * h.n_src, N2 = (size_t)h.n_img * h.n_img;
  h.src = c.take<float>(B * n2);
  h.fld = c.take<float>(B * n2);
  h.F = c.take<float2>(B * n2);
  h.tmp = c.take<float2>(B * n2);
  h.knots = c.take<float>((size_t)B * 4 * K);
  h.kdbg = c.take<float>((size_t)B * 4 * K);
  h.sel = c.take<int>((size_t)B * 4 * K);
  h.stdv = c.take<double>((size_t)B * 4);
  h.dp = c.take<float>((size_t)B * 2 * K);
  h.u = c.take<float>(B * N2);
  h.r = c.take<float>(B * N2);
  h.ubar = c.take<float>(B * N2);
  h.sbar = c.take<float>(B * n2);
  h.kbar = c.take<float>((size_t)B * h.ray_tiles * 4 * K);
  h.lpart = c.take<double>((size_t)B * h.ray_tiles * h.n_lens);
  h.c2part = c.take<double>((size_t)B * h.psf_tiles * 2);
  h.st = c.take<uint32_t>((size_t)B * 4);
  return c.off + 256;
}

// observation and mask-dependent buffers
size_t carve_observation(SysDev& h, int B, int M, char* base) {
  Carve c{base};
  const size_t N2 = (size_t)h.n_img * h.n_img, k2 = (size_t)h.psf_k * h.psf_k;
  h.image = c.take<float>(N2);
  h.inv_var = c.take<float>(N2);
  h.psf_flip = c.take<float>(k2);
  h.psf = c.take<float>(k2);
  h.mask = c.take<uint8_t>(N2);
  h.mask_idx = c.take<int>(M > 0 ? M : 1);
  h.rank_j = c.take<int>(K);
  h.rank_t = c.take<double>(K);
  h.zbuf = c.take<float>((size_t)B * 2 * (M > 0 ? M : 1));
  h.cand = c.take<unsigned long long>((size_t)B * 2 * (M > 0 ? M : 1));
  return c.off + 256;
}

}  // namespace

extern "C" {

int32_t rtu_n_lens(const rtu_geometry* g) {
  return g ? RTU_N_LENS_BASE + RTU_N_PER_SUB * g->n_sub_max : 0;
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
  if (hipMalloc(&p->pool, bytes) != hipSuccess) {
    delete p;
    return RTU_ENOMEM;
  }
  carve_workspace(p->h, max_batch, p->pool);
  *out = p;
  return RTU_OK;
}

int rtu_plan_destroy(rtu_plan p) {
  if (!p) return RTU_EINVAL;
  hipSetDevice(p->device);
  hipDeviceSynchronize();
  if (p->pool) hipFree(p->pool);
  if (p->obs_pool) hipFree(p->obs_pool);
  delete p;
  return RTU_OK;
}

int rtu_set_observation(rtu_plan p, const float* image, const float* noise_sigma, const float* psf,
                        const uint8_t* arc_mask) {
  if (!p || !image || !noise_sigma || !psf || !arc_mask) return RTU_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess) return RTU_EHIP;
  const int N = p->g.n_img, KP = p->g.psf_size;
  const size_t N2 = (size_t)N * N;
  std::vector<int> idx;
  for (size_t q = 0; q < N2; ++q)
    if (arc_mask[q]) idx.push_back((int)q);
  const int M = (int)idx.size();
  // quantile ranks of the Chebyshev nodes: h_k = (M-1) u_k in FP64
  int rj[K];
  double rt[K];
  for (int k = 0; k < K; ++k) {
    const double u = 0.5 * (1.0 - cos((2.0 * (k + 1) - 1.0) * M_PI / (2.0 * K)));
    const double hh = (double)(M > 0 ? M - 1 : 0) * u;
    const double fl = floor(hh);
    rj[k] = (int)fl;
    rt[k] = hh - fl;
  }
  std::vector<float> iv(N2), flip((size_t)KP * KP);
  for (size_t q = 0; q < N2; ++q) iv[q] = 1.f / (noise_sigma[q] * noise_sigma[q]);
  for (int a = 0; a < KP; ++a)
    for (int b = 0; b < KP; ++b) flip[(size_t)a * KP + b] = psf[(size_t)(KP - 1 - a) * KP + (KP - 1 - b)];
  SysDev h = p->h;
  const size_t bytes = carve_observation(h, p->max_batch, M, nullptr);
  if (bytes > p->obs_bytes) {
    hipDeviceSynchronize();
    if (p->obs_pool) hipFree(p->obs_pool);
    p->obs_pool = nullptr;
    p->obs_bytes = 0;
    if (hipMalloc(&p->obs_pool, bytes) != hipSuccess) return RTU_ENOMEM;
    p->obs_bytes = bytes;
  }
  carve_observation(h, p->max_batch, M, p->obs_pool);
  hipError_t e = hipSuccess;
  auto cp = [&](const void* dst, const void* src, size_t n) {
    if (e == hipSuccess && n) e = hipMemcpy(const_cast<void*>(dst), src, n, hipMemcpyHostToDevice);
  };
  cp(h.image, image, N2 * 4);
  cp(h.inv_var, iv.data(), N2 * 4);
  cp(h.psf_flip, flip.data(), (size_t)KP * KP * 4);
  cp(h.psf, psf, (size_t)KP * KP * 4);
  cp(h.mask, arc_mask, N2);
  cp(h.mask_idx, idx.data(), (size_t)M * 4);
  cp(h.rank_j, rj, sizeof(rj));
  cp(h.rank_t, rt, sizeof(rt));
  if (e != hipSuccess) return RTU_EHIP;
  h.M = M;
  p->h = h;
  p->M = M;
  return RTU_OK;
}

int32_t rtu_masked_count(rtu_plan p) { return p ? p->M : -1; }

int rtu_loss_grad(rtu_plan p, int32_t batch, const float* lens_params, const int32_t* n_sub,
                  const float* ps_params, const float* latent, double* loss, double* chi2_mask,
                  float* grad_lens, float* grad_ps, float* grad_latent, float* model_image,
                  uint32_t* status, void* stream) {
  if (!p) return RTU_EINVAL;
  if (p->M < 0) return RTU_ESTATE;
  if (batch < 1) return RTU_EINVAL;
  if (batch > p->max_batch) return RTU_EBATCH;
  if (!lens_params || !ps_params || !latent || !loss || !status) return RTU_EINVAL;
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
  if (launch_prep(h, batch, s) != hipSuccess) return RTU_EHIP;
  if (launch_rays_fwd(h, batch, s) != hipSuccess) return RTU_EHIP;
  if (launch_psf(h, batch, false, s) != hipSuccess) return RTU_EHIP;
  if (h.want_grad) {
    if (launch_psf(h, batch, true, s) != hipSuccess) return RTU_EHIP;
    if (launch_rays_adj(h, batch, s) != hipSuccess) return RTU_EHIP;
  }
  if (launch_post(h, batch, s) != hipSuccess) return RTU_EHIP;
  p->last = h;
  p->have_last = true;
  return RTU_OK;
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
    default: return RTU_EINVAL;
  }
  if (bytes < need) return RTU_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(s) != hipSuccess) return RTU_EHIP;
  if (hipMemcpy(host_dst, src, need, hipMemcpyDeviceToHost) != hipSuccess) return RTU_EHIP;
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
    default: return "unknown error";
  }
}

}  // extern "C"
