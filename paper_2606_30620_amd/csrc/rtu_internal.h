// Internal layout shared by the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rtu.h"

namespace rtu {

constexpr int K = RTU_K_NODES;          // Chebyshev nodes (degree 21 + 1)
constexpr int RAY_TILE = 16;            // ray kernels: 16x16 pixel tile per workgroup
constexpr int RAY_THREADS = RAY_TILE * RAY_TILE;
constexpr int PSF_TW = 64;              // PSF kernels: 64 x 16 output tile,
constexpr int PSF_TH = 16;              // 256 threads x 4 columns each
constexpr int PSF_THREADS = 256;
constexpr int PREP_THREADS = 1024;      // quantile selection and FFT workgroups
constexpr int HIST_BINS = 4096;         // first-level histogram of the selection
constexpr int SEL_LDS_CAP = 3072;       // candidates kept in LDS (else global scratch)
constexpr int GRID_LDS_MAX = 64;        // n_src <= this: source grid staged in LDS
constexpr int FFT_LDS_FLOAT2 = 4224;    // FFT chunk buffer (float2) = 33 KB
constexpr int KBAR = 4 * K;             // per axis pair: dX[K], dS[K]  (x: 0..2K, y: 2K..4K)

// Everything a kernel needs about one lens system and the samples of a call.
// Sample b of a per-sample array starts at base + b * (its per-sample size).
struct SysDev {
  // geometry
  int n_img, ss, n_src, log2_src, psf_k, n_sub_max, n_lens, M;
  float pix, tau, inv_ss2;
  int ray_tx, ray_tiles;      // 16x16 ray tiles per side / per sample
  int psf_tx, psf_tiles;      // 64x16 PSF tiles along x / per sample
  int want_grad, batch;
  // observation (owned by the plan)
  const float* image;         // [N*N]
  const float* inv_var;       // [N*N] 1/sigma^2
  const float* psf_flip;      // [K*K] PSF rotated by 180 degrees (forward correlation)
  const float* psf;           // [K*K] PSF as given (adjoint correlation)
  const uint8_t* mask;        // [N*N]
  const int* mask_idx;        // [M] row-major pixel index of each masked pixel
  const int* rank_j;          // [K] floor((M-1) u_k)
  const double* rank_t;       // [K] (M-1) u_k - rank_j
  // per-call inputs
  const float* lens;          // [B][n_lens]
  const int* n_sub;           // [B] or null
  const float* ps;            // [B][4]
  const float* latent;        // [B][n_src^2]
  // per-call outputs
  double* loss;               // [B]
  double* chi2m;              // [B] or null
  float* g_lens;              // [B][n_lens] or null
  float* g_ps;                // [B][4] or null
  float* g_lat;               // [B][n_src^2] or null
  float* model;               // [B][N^2] or null
  uint32_t* status;           // [B]
  // workspace (owned by the plan)
  float* src;                 // [B][n^2] source brightness s
  float* fld;                 // [B][n^2] GP field f
  float2* F;                  // [B][n^2] DFT of the latent
  float2* tmp;                // [B][n^2] FFT scratch
  float* zbuf;                // [B][2][M] masked-ray beta per axis
  unsigned long long* cand;   // [B][2][M] selection candidates (slow path)
  float* knots;               // [B][2][2][K] per axis: X_k, S_k in beta units
  float* kdbg;                // [B][2][2][K] per axis: X_k, S_k standardised
  int* sel;                   // [B][2][2][K] per axis: ray index at rank j, j+1
  double* stdv;               // [B][4] mean x, mean y, s
  float* dp;                  // [B][2][K] p'(u_k) in beta units; <= 0: clamped
  float* u;                   // [B][N^2] sub-ray mean image
  float* r;                   // [B][N^2] (m - d)/sigma^2
  float* ubar;                // [B][N^2] d loss / d u
  float* sbar;                // [B][n^2] d loss / d s
  float* kbar;                // [B][ray_tiles][4K] per-tile dX, dS partials
  double* lpart;              // [B][ray_tiles][n_lens] per-tile lens-gradient partials
  double* c2part;             // [B][psf_tiles][2] per-tile chi^2 partials (all, mask)
  uint32_t* st;               // [B][4] status words of the stages
};

// One stochastic variational fit: guide, Adam state and per-sample buffers.
struct FitDev {
  int S, dim, n_lens, n_src2;
  float lr;
  uint32_t seed_lo, seed_hi;
  double elbo_const;          // data and prior normalisation + guide entropy constant
  float *mu, *rho, *m_mu, *v_mu, *m_rho, *v_rho;   // [dim]
  float *z_lens, *z_ps, *z_lat;                    // [S][...] samples (evaluation inputs)
  float *g_lens, *g_ps, *g_lat;                    // [S][...] gradients (evaluation outputs)
  double* loss;               // [S]
  double* chi2m;              // [S]
  uint32_t* status;           // [S]
  int* n_sub;                 // [S]
  double* trace;              // [max_steps] ELBO per step
};

// kernel launchers (rtu_kernels.hip)
hipError_t upload_constants();
hipError_t launch_prep(const SysDev& h, int batch, hipStream_t s);
hipError_t launch_rays_fwd(const SysDev& h, int batch, hipStream_t s);
hipError_t launch_psf(const SysDev& h, int batch, bool adjoint, hipStream_t s);
hipError_t launch_rays_adj(const SysDev& h, int batch, hipStream_t s);
hipError_t launch_post(const SysDev& h, int batch, hipStream_t s);
// fit kernels (rtu_fit.hip)
hipError_t launch_sample(const FitDev& F, const float* eps, int step, hipStream_t s);
hipError_t launch_adam(const FitDev& F, const float* eps, int step, int t, hipStream_t s);

}  // namespace rtu
