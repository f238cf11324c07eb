// gfx950 kernels of the stochastic variational fit (Sec. 4): reparameterised
// sampling of the guide, the ELBO estimate, and the Adam update.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rtu_device.h"
#include "rtu_internal.h"

namespace rtu {

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011): 10 rounds of the
// multiply-xor bijection on a 128-bit counter under a 64-bit key.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += W0;
    k.y += W1;
  }
  return c;
}

// Standard normal draws of samples 4c .. 4c + 3 of (step, parameter): one
// Philox block (counter: parameter, c, step, a constant) gives four 32-bit
// uniforms, and Box-Muller turns each pair into two normals (cosine and sine
// branch).
__device__ __forceinline__ void normal_draw4(const FitDev& F, int step, int c, int i, float (&z)[4]) {
  const uint4 r = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)c, (uint32_t)step, 0x52545547u),
                                make_uint2(F.seed_lo, F.seed_hi));
  const float k = 2.3283064365386963e-10f;          // 2^-32
  const float ra = sqrtf(-2.f * __logf(((float)r.x + 0.5f) * k)), ta = 6.283185307179586f * (float)r.y * k;
  const float rb = sqrtf(-2.f * __logf(((float)r.z + 0.5f) * k)), tb = 6.283185307179586f * (float)r.w * k;
  z[0] = ra * __cosf(ta); z[1] = ra * __sinf(ta);
  z[2] = rb * __cosf(tb); z[3] = rb * __sinf(tb);
}
__device__ __forceinline__ float normal_draw(const FitDev& F, int step, int s, int i) {
  float z[4];
  normal_draw4(F, step, s >> 2, i, z);
  const int k = s & 3;
  return k == 0 ? z[0] : (k == 1 ? z[1] : (k == 2 ? z[2] : z[3]));
}

__device__ __forceinline__ float eps_at(const FitDev& F, const float* eps, int step, int s, int i) {
  return eps ? eps[(size_t)s * F.dim + i] : normal_draw(F, step, s, i);
}

__device__ __forceinline__ bool is_log(const FitDev& F, int i) {
  return i < F.n_lens + 4 && ((F.log_mask[i >> 5] >> (i & 31)) & 1u);
}

// z_s = mu + exp(rho) eps_s (z = exp of that for a log-space parameter),
// scattered into the plan's per-sample inputs; the draw is kept for the Adam
// update of rho.  mu, sig = exp(rho) of parameter i.
__device__ __forceinline__ void sample_store(const FitDev& F, int s, int i, float mu, float sig, float e) {
  F.eps_s[(size_t)s * F.dim + i] = e;
  float z = mu + sig * e;
  if (is_log(F, i)) z = __expf(z);
  if (i < F.n_lens) F.z_lens[(size_t)s * F.n_lens + i] = z;
  else if (i < F.n_lens + 4) F.z_ps[(size_t)s * 4 + (i - F.n_lens)] = z;
  else F.z_lat[(size_t)s * F.n_src2 + (i - F.n_lens - 4)] = z;
}

// d loss / d u of sample s: the evaluation's gradient, times z for a
// log-space parameter (z = exp(u))
__device__ __forceinline__ float grad_at(const FitDev& F, int s, int i) {
  if (i < F.n_lens) {
    const float g = F.g_lens[(size_t)s * F.n_lens + i];
    return is_log(F, i) ? g * F.z_lens[(size_t)s * F.n_lens + i] : g;
  }
  if (i < F.n_lens + 4) {
    const float g = F.g_ps[(size_t)s * 4 + (i - F.n_lens)];
    return is_log(F, i) ? g * F.z_ps[(size_t)s * 4 + (i - F.n_lens)] : g;
  }
  return F.g_lat[(size_t)s * F.n_src2 + (i - F.n_lens - 4)];
}

// Adam on (mu, rho) with the gradient of -ELBO:
//   d/dmu_i  = mean_s g_si,   d/drho_i = mean_s g_si exp(rho_i) eps_si - 1
// A workgroup takes ADAM_P parameters; its G = blockDim / ADAM_P groups of
// threads (as many as the launch's largest sample count needs, at most 16)
// each sum every G-th sample of a parameter, and group 0 adds the group sums in
// group order (so that more workgroups share the memory latency of the
// S gradient and draw loads) and leaves the new mu and exp(rho) in nmu,
// nsig.  Called by every thread of the workgroup.
__device__ __forceinline__ void adam_body(const FitDev& F, int t, int i, int g, float* red, float* nmu,
                                          float* nsig) {
  const int p = threadIdx.x % ADAM_P, G = blockDim.x / ADAM_P;
  float gm = 0.f, gr = 0.f;
  if (i < F.dim) {
#pragma unroll 4
    for (int s = g; s < F.S; s += G) {
      const float gs = grad_at(F, s, i);
      gm += gs;
      gr += gs * F.eps_s[(size_t)s * F.dim + i];
    }
  }
  red[g * ADAM_P + p] = gm;
  red[(G + g) * ADAM_P + p] = gr;
  __syncthreads();
  if (g != 0 || i >= F.dim) return;
  gm = red[p];
  gr = red[G * ADAM_P + p];
  for (int k = 1; k < G; ++k) {
    gm += red[k * ADAM_P + p];
    gr += red[(G + k) * ADAM_P + p];
  }
  const float sig = __expf(F.rho[i]);
  const float invS = 1.f / (float)F.S;
  gm *= invS;
  gr = gr * invS * sig - 1.f;
  const float b1 = 0.9f, b2 = 0.999f, e = 1e-8f;
  const float c1 = 1.f / (1.f - powf(b1, (float)t)), c2 = 1.f / (1.f - powf(b2, (float)t));
  float m = b1 * F.m_mu[i] + (1.f - b1) * gm;
  float v = b2 * F.v_mu[i] + (1.f - b2) * gm * gm;
  F.m_mu[i] = m;
  F.v_mu[i] = v;
  F.mu[i] -= F.lr * (m * c1) / (sqrtf(v * c2) + e);
  m = b1 * F.m_rho[i] + (1.f - b1) * gr;
  v = b2 * F.v_rho[i] + (1.f - b2) * gr * gr;
  F.m_rho[i] = m;
  F.v_rho[i] = v;
  const float rho = F.rho[i] - F.lr * (m * c1) / (sqrtf(v * c2) + e);
  F.rho[i] = rho;
  nmu[p] = F.mu[i];
  nsig[p] = __expf(rho);
}

// ---- shared launches over many fits (serving); step = round - round0
__device__ __forceinline__ bool fit_step(const FitDev& F, int round, int& step) {
  step = round - F.round0;
  return step >= 0 && step < F.nsteps;
}

// rho_part[step & 1][j]: the sum of rho over parameter block j of ADAM_P at
// the time the samples of `step` were drawn (the ELBO's entropy term).
__device__ __forceinline__ double* rho_part_of(const FitDev& F, int step) {
  return F.rho_part + (size_t)(step & 1) * ((F.dim + ADAM_P - 1) / ADAM_P);
}

// The samples of a step: a fit's first step, one after a restored state, and
// every step with given draws.  (With Philox draws the Adam update of a step
// draws the next step's samples.)  The blocks of sample 0 also write the
// rho sums of their ADAM_P-blocks (one wave each).
__global__ void __launch_bounds__(FIT_THREADS) kf_sample(const FitDev* __restrict__ fits,
                                                         const Task* __restrict__ tasks, int round,
                                                         const float* eps) {
  const Task t = tasks[blockIdx.x];      // x fit, y parameter block, z sample
  const FitDev& F = fits[t.x];
  int step;
  if (!fit_step(F, round, step)) return;
  const int i = t.y * FIT_THREADS + threadIdx.x;
  if (i < F.dim) sample_store(F, t.z, i, F.mu[i], __expf(F.rho[i]), eps_at(F, eps, step, t.z, i));
  if (t.z == 0) {
    static_assert(FIT_THREADS % ADAM_P == 0 && ADAM_P == 64, "one wave per rho block");
    const double r = wave_sum(i < F.dim ? (double)F.rho[i] : 0.0);
    const int j = i / ADAM_P;
    if ((threadIdx.x & 63) == 0 && j * ADAM_P < F.dim) rho_part_of(F, step)[j] = r;
  }
}

// Adam; with draw set (Philox draws) each block then draws the next step's
// samples of its parameters from the updated guide and their rho sum.  Block
// 0 of each fit also writes the ELBO of this step from the rho sums taken
// when this step's samples were drawn, the losses and the status words, each
// summed in a fixed order.
__global__ void __launch_bounds__(ADAM_THREADS) kf_adam(const FitDev* __restrict__ fits,
                                                        const Task* __restrict__ tasks, int round, int draw) {
  __shared__ float red[2 * ADAM_THREADS];
  __shared__ float nmu[ADAM_P], nsig[ADAM_P];
  const Task t = tasks[blockIdx.x];      // x fit, y block of ADAM_P parameters
  const FitDev& F = fits[t.x];
  int step;
  if (!fit_step(F, round, step)) return;
  const int p = threadIdx.x % ADAM_P, g = threadIdx.x / ADAM_P, i = t.y * ADAM_P + p;
  adam_body(F, step + 1, i, g, red, nmu, nsig);
  __syncthreads();
  if (draw) {
    if (i < F.dim)
      for (int c = g; 4 * c < F.S; c += (int)(blockDim.x / ADAM_P)) {   // four samples per Philox block
        float z[4];
        normal_draw4(F, step + 1, c, i, z);
        for (int k = 0; k < 4 && 4 * c + k < F.S; ++k) sample_store(F, 4 * c + k, i, nmu[p], nsig[p], z[k]);
      }
    if (g == 0) {
      const double r = wave_sum(i < F.dim ? (double)F.rho[i] : 0.0);
      if (p == 0) rho_part_of(F, step + 1)[t.y] = r;
    }
  }
  if (t.y != 0 || threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  const int nblk = (F.dim + ADAM_P - 1) / ADAM_P;
  const double* rp = rho_part_of(F, step);
  double a = 0.0, ls = 0.0;
  uint32_t st = 0;
  for (int j0 = 0; j0 < nblk; j0 += 64) a += wave_sum(j0 + lane < nblk ? rp[j0 + lane] : 0.0);
  for (int s0 = 0; s0 < F.S; s0 += 64) {
    ls += wave_sum(s0 + lane < F.S ? F.loss[s0 + lane] : 0.0);
    const int v = s0 + lane < F.S ? (int)F.status[s0 + lane] : 0;
    st |= (uint32_t)wave_reduce(v, [](int x, int y) { return x | y; });
  }
  if (lane == 0) {
    F.trace[step] = -ls / (double)F.S + F.elbo_const + a;
    if (F.status_acc) F.status_acc[0] |= st;
  }
}

hipError_t launch_fleet_fit_stage(const FleetLaunch& L, int stage, int round, const float* eps, hipStream_t s) {
  if (stage == RTU_STAGE_SAMPLE) {
    if (L.n_sample) hipLaunchKernelGGL(kf_sample, dim3(L.n_sample), dim3(FIT_THREADS), 0, s, L.fit, L.t_sample,
                                      round, eps);
  } else if (stage == RTU_STAGE_ADAM) {
    if (L.n_param)
      hipLaunchKernelGGL(kf_adam, dim3(L.n_param), dim3(L.adam_threads), 0, s, L.fit, L.t_param, round,
                         eps ? 0 : 1);
  }
  return hipGetLastError();
}

}  // namespace rtu
