// Internal layout shared by the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/rtu.h"

namespace rtu {

constexpr int K = RTU_K_NODES;          // Chebyshev nodes (degree 21 + 1)
// ray kernels: a 16 x 16 pixel tile per workgroup, one pixel per thread, each
// wave an 8 x 8 quarter of it (past an image edge at a multiple of 8 a whole
// wave is outside and exits, instead of half the lanes of every wave idling)
constexpr int RAY_TILE = 16;
constexpr int RAY_THREADS = RAY_TILE * RAY_TILE;
constexpr int PSF_TW = 64;              // PSF kernels: 64 x 16 output tile,
constexpr int PSF_TH = 16;              // 256 threads x 4 columns each
constexpr int PSF_THREADS = 256;
constexpr int ST_WORDS = 8;
constexpr int PREP_THREADS = 512;       // quantile selection and FFT workgroups,
constexpr int PREP_THREADS_WIDE = 1024; // twice as wide for masks of PREP_WIDE_M rays or more
constexpr int PREP_WIDE_M = 12000;
constexpr int POST_THREADS = 512;       // per-sample adjoint workgroups
// Masks of MR_MIN_M rays or more are shot before the selection by a launch
// of its own, MR_CHUNK rays per workgroup of MR_THREADS, over many CUs
// (the selection workgroup of a sample runs on one CU); the selection
// then sums the chunks' moments and ranges in chunk order.
constexpr int MR_THREADS = 256;
constexpr int MR_CHUNK = 1024;
constexpr int MR_MIN_M = 8192;
inline int mr_chunks(int M) { return M >= MR_MIN_M ? (M + MR_CHUNK - 1) / MR_CHUNK : 0; }
constexpr int GRID_LDS_MAX = 64;        // n_src <= this: the ray adjoint keeps d loss / d s in LDS
constexpr int KBAR = 4 * K;
// GP transforms of source grids of at least GP_SPLIT_N per side run as three
// line passes (rows, columns, rows) through the workspace, each pass a launch
// of GP_LINES lines per workgroup
constexpr int GP_LINES = 16;
constexpr int GP_SPLIT_N = 256;
constexpr int GP_THREADS = 256;
__host__ __device__ constexpr bool gp_split(int n) { return n >= GP_SPLIT_N; }
// Prep workgroup size for a mask of M rays (0: not known on the host) and an
// n_src grid.  The selection's passes over the rays (histogram, gather, and
// the shooting below MR_MIN_M) shorten with more threads only when each
// thread has many rays, and the GP role's one-workgroup transform only from
// 128 x 128 on; otherwise the barriers of sixteen waves cost more than the
// passes save.
inline int prep_threads(int M, int n_src) {
  return M >= PREP_WIDE_M || (n_src >= 128 && !gp_split(n_src)) ? PREP_THREADS_WIDE : PREP_THREADS;
}
constexpr int FIT_THREADS = 256;        // fit kernels: sampling blocks of 256 parameters,
constexpr int ADAM_P = 64;              // Adam blocks of 64 parameters
constexpr int ADAM_THREADS = 1024;      // Adam blocks: ADAM_P parameters x up to 16 sample groups

// PSF on the matrix cores: K-steps of 4 per PSF row for 16 output columns
// (at least 15 + KP window columns), the padded weight-row length, and the
// LDS row stride of the input tile (covers the halo and the last wave's last
// step; 4 mod 8, so that one MFMA operand's 16 rows x 4 columns fall in
// distinct banks).
__host__ __device__ constexpr int psf_nk(int KP) { return (15 + KP + 3) / 4; }
__host__ __device__ constexpr int psf_ws(int KP) { return 4 * psf_nk(KP) + 16; }
// separable PSF: LDS row stride of the input tile (its 64 + KP - 1 columns
// after a shift of up to 3 that aligns them to float4 groups)
__host__ __device__ constexpr int psf_sep_stride(int KP) { return (PSF_TW + KP - 1 + 6) & ~3; }
__host__ __device__ constexpr int psf_row_stride(int KP) {
  return (PSF_TW - 16 + 4 * psf_nk(KP)) % 8 == 4 ? PSF_TW - 16 + 4 * psf_nk(KP) : PSF_TW - 12 + 4 * psf_nk(KP);
}             // per axis pair: dX[K], dS[K]  (x: 0..2K, y: 2K..4K)

// Pixel (i, j)'s centre ((j - (N-1)/2) d, (i - (N-1)/2) d), the same FP32
// arithmetic on the host and the device.
__host__ __device__ inline float2 pixel_centre(int p, int N, float pix) {
  const int i = p / N, j = p - i * N;
  return make_float2(((float)j - 0.5f * (float)(N - 1)) * pix, ((float)i - 0.5f * (float)(N - 1)) * pix);
}

// The order statistics the selection needs: ranks floor(h_k) and floor(h_k) + 1
// of the 22 nodes (clamped to [0, M - 1]).  Each sequence is non-decreasing,
// but with few masked rays neighbouring nodes share floor(h_k), so
// floor(h_k) + 1 can exceed floor(h_{k+1}); the selections take the distinct
// ranks in ascending order.  out[0, n): those ranks (the rest 0x7fffffff);
// out[2K + t]: the place of rank t (node t / 2, + (t & 1)) in that list;
// out[4K] = n.  It depends on the mask only, so it is made once per
// observation.
__host__ __device__ inline void target_list(const int* rank_j, int M, int* out) {
  int r[2 * K];
  for (int t = 0; t < 2 * K; ++t) {
    const int v = rank_j[t >> 1] + (t & 1);
    r[t] = v < 0 ? 0 : (v > M - 1 ? M - 1 : v);
  }
  int n = 0;
  for (int t = 0; t < 2 * K; ++t) out[t] = 0x7fffffff;
  for (int t = 0; t < 2 * K; ++t) {
    bool first = true;
    for (int s = 0; s < t; ++s) first = first && r[s] != r[t];
    int below = 0;
    for (int s = 0; s < 2 * K; ++s) {
      bool fs = true;
      for (int u = 0; u < s; ++u) fs = fs && r[u] != r[s];
      below += (fs && r[s] < r[t]) ? 1 : 0;
    }
    if (first) { out[below] = r[t]; ++n; }
    out[2 * K + t] = below;
  }
  out[4 * K] = n;
}

// Per-sample tables of the two smoothed-CDF splines, in the layout the ray
// kernels keep in LDS; built once per sample by the selection workgroups (each
// writes its axis).  For axis ax and interval k (0: below the first knot, K:
// above the last; else [X_{k-1}, X_k)): the local coordinate
// t = (z - ct.x) ct.y and the grid coordinate T = n g - 1/2 =
// ((cq.w t + cq.z) t + cq.y) t + cq.x.
struct KnotTab {
  float4 cq[2][K + 1];
  float2 ct[2][K + 1];
  float2 kr[2][K + 1];  // interval k as [kr.x, kr.y), with -inf / +inf at the ends
  float xs[2][32];      // knots, then +inf (branch-free search)
  float X[2][K], Sl[2][K], ih[2][K], dp[2][K];
  float du[K];          // u_{l+1} - u_l (0 for l = K-1)
  float zr[2][2];       // per axis: the z below which T < -2.25 and above which
                        // T > n + 1.25 (the affine end pieces; -inf / +inf if
                        // their slope is not positive)
  float pad[2];
};
static_assert(sizeof(KnotTab) % 16 == 0, "KnotTab is copied as float4");

// Per-sample constants of the singular isothermal ellipsoid (eq. A1 at slope
// 2) and the external shear, made once per sample by the selection workgroup
// of axis 0 and read by the ray kernels.
struct Sie {
  float the, x0, y0, g1, g2;
  float c, s;        // cos, sin of the position angle phi = atan2(e2, e1)/2
  float q, f, P;     // axis ratio, f = sqrt(1-q^2), P = theta_E sqrt(q)
  float q2;          // q^2
  float invf;        // 1/f
  float e1, e2, e;
  bool round;        // e < E_ROUND: the angle-free gradient
  float cpe, spe;    // c/(1+e), s/(1+e)
  float cq, sq;      // c q, s q
  float im2f;        // 1/(1+e)^2
  float jb, gam;     // |theta_E| / sqrt(q); shear modulus gamma
};

// Everything a kernel needs about one lens system and the samples of a call.
// Sample b of a per-sample array starts at base + b * (its per-sample size).
// Moments and ranges of one chunk of masked rays (both axes): the (weighted)
// sums of beta_x, beta_y and their squares, the finite value range and the
// order-key range per axis, the uniform grid's extreme keys (x min, x max,
// y min, y max).
struct MRayPart {
  double s[4];
  float vmin[2], vmax[2];
  unsigned umin[2], umax[2];
  unsigned long long k[4];
};

struct SysDev {
  // geometry
  int n_img, ss, n_src, log2_src, psf_k, n_sub_max, n_lens, M;
  int n_gauss, light_off;     // lens-light Gaussians and their offset in the lens vector
  float pix, tau, inv_ss2;
  int ray_tx, ray_tiles;      // 16x16 ray tiles along x / per sample
  int psf_tx, psf_tiles;      // 64x16 PSF tiles along x / per sample
  int want_grad, batch;
  int round0, nsteps;         // serving: rounds [round0, round0 + nsteps) are this system's steps
  int lds_adj;                // the ray adjoint keeps d loss / d s in LDS (1) or adds to global memory (0)
  int adj_wcap;               // global mode: cells of the per-tile LDS window of d loss / d s
  int sel_radix;              // quantile selection: always the radix select (1)
  int uniform;                // uniform grid on the masked rays' square box (1) instead of the RTU grid
  int epl;                    // main deflector: EPL with free slope (1) or SIE (0)
  int lens_base;              // lens parameters before the subhaloes: 7 (SIE), 8 (EPL)
  // observation (owned by the plan)
  const float* image;         // [N*N]
  const float* inv_var;       // [N*N] 1/sigma^2
  const float* psf_flip;      // [KP][psf_ws(KP)] PSF rotated by 180 degrees (forward correlation),
                              // each row zero-padded: W[a][c] at [a][c + 15]
  const float* psf;           // [KP][psf_ws(KP)] PSF as given (adjoint correlation), padded the same way
  const float* psf_sep;       // [4][KP] for a rank-one PSF W[a][c] = u[a] v[c]: u, v of the forward
                              // (flipped) correlation, then u, v of the adjoint one
  int psf_rank1;              // the PSF is rank one (to FP32 rounding): the separable PSF kernel
  const int* obs_dyn;         // null, or an observation prepared on the device: [0] M, [1] psf_rank1
                              // (these then replace the two fields above)
  const uint8_t* mask;        // [N*N]
  const int* mask_idx;        // [M] row-major pixel index of each masked pixel
  const float2* mask_xy;      // [M] its image-plane position (the pixel centre)
  const int* rank_j;          // [K] floor((M-1) u_k)
  const double* rank_t;       // [K] (M-1) u_k - rank_j
  const int* tsel;            // [4K + 1] the selection's targets (target_list)
  // weighted RTU grid (ray_w non-null): per masked ray its weight, the total
  // W, per node floor((W-1) u_k) and its fraction, and sort scratch
  const float* ray_w;         // [M]
  double wsum;
  const double* wr0;          // [K]
  const double* wt;           // [K]
  uint2* wsort;               // [B][2 axes][2][M] (order key, ray index)
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
  float* srcp;                // [B][(n+2)^2] s with a one-cell zero border (corner reads need no bounds checks)
  KnotTab* ktab;              // [B] spline tables for the ray kernels
  Sie* sie;                   // [B] SIE + shear constants for the ray kernels
  float* fld;                 // [B][n^2] GP field f
  float2* F;                  // [B][n^2] DFT of the latent
  float2* tmp;                // [B][n^2] FFT scratch
  double* gpp;                // [B][n / GP_LINES][4] split GP adjoint: spectrum-gradient partials per workgroup
  float* zbuf;                // [B][2][M] masked-ray beta per axis
  MRayPart* mrp;              // [B][mr_nchunk] chunk partials of the masked-ray launch
  int mr_nchunk;               // chunks of that launch per sample (0: the selection shoots the rays)
  float* knots;               // [B][2][2][K] per axis: X_k, S_k in beta units
  float* kdbg;                // [B][2][2][K] per axis: X_k, S_k standardised
  int* sel;                   // [B][2][2][K] per axis: ray index at rank j, j+1
  double* stdv;               // [B][4] mean x, mean y, s, M (uniform grid: lo_x, lo_y, L,
                              // the axis whose range is L)
  float* dp;                  // [B][2][K] p'(u_k) in beta units; <= 0: clamped
  float* u;                   // [B][N^2] sub-ray mean image
  float* r;                   // [B][N^2] (m - d)/sigma^2
  float* ubar;                // [B][N^2] d loss / d u
  double* sbar;               // [B][n^2] d loss / d s (FP64 accumulation: order-independent to FP32 rounding)
  double* kbar;               // [B][ray_tiles][4K] per-tile dX, dS partials
  int4* tbox;                 // [B][ray_tiles][4 waves] source cells the forward's sub-rays fell in:
                              // (min row, min column, max row, max column) of the cell's lower corner
  double* lpart;              // [B][ray_tiles][4 waves][n_lens + 2] per-wave raw lens-gradient partials,
                              // then the number of the wave's sub-rays on the grid
  double* c2part;             // [B][psf_tiles][2] per-tile chi^2 partials (all, mask)
  uint32_t* st;               // [B][ST_WORDS] status words: selection x, y; parameter domain
};

// One stochastic variational fit: guide, Adam state and per-sample buffers.
struct FitDev {
  int S, dim, n_lens, n_src2;
  int round0, nsteps;         // serving: step = round - round0, active while < nsteps
  float lr;
  uint32_t seed_lo, seed_hi;
  uint32_t log_mask[RTU_LOG_MASK_WORDS];   // lens parameter i has a log-space guide if bit i is set
  double elbo_const;          // data and prior normalisation + guide entropy constant
  float *mu, *rho, *m_mu, *v_mu, *m_rho, *v_rho;   // [dim]
  float *z_lens, *z_ps, *z_lat;                    // [S][...] samples (evaluation inputs)
  float *g_lens, *g_ps, *g_lat;                    // [S][...] gradients (evaluation outputs)
  float* eps_s;                                    // [S][dim] this step's standard-normal draws
  double* loss;               // [S]
  double* chi2m;              // [S]
  uint32_t* status;           // [S]
  int* n_sub;                 // [S]
  double* trace;              // [max_steps] ELBO per step
  uint32_t* status_acc;       // [1] OR of every sample status over all steps
  double* rho_part;           // [ceil(dim / 256)] per parameter block: the sum of rho at sampling time
};

// One work item of a shared (serving) launch: x = system/fit slot,
// y = sample (or parameter block), z = tile / role / sample.
using Task = int4;

// kernel launchers (rtu_kernels.hip)
hipError_t upload_constants();
hipError_t launch_prep(const SysDev& h, int batch, hipStream_t s);
hipError_t launch_rays_fwd(const SysDev& h, int batch, hipStream_t s);
hipError_t launch_psf(const SysDev& h, int batch, bool adjoint, hipStream_t s);
hipError_t launch_rays_adj(const SysDev& h, int batch, hipStream_t s);
hipError_t launch_post(const SysDev& h, int batch, hipStream_t s);
// the observation tables of h (inv_var, PSF rows, rank-one factors, masked
// pixels, ranks) prepared on the device from the raw observation, M and the
// rank-one flag written to dyn[0], dyn[1]
hipError_t launch_observe(const SysDev& h, const float* noise_sigma, const float* psf, int* dyn, hipStream_t s);
// fit kernels (rtu_fit.hip)

// host helpers shared by plans, fits and the serving fleet (rtu_runtime.hip)
struct ObsHost {
  std::vector<int> idx;       // masked pixels, row-major
  std::vector<float2> xy;     // their pixel centres
  int rank_j[K];
  double rank_t[K];
  int tsel[4 * K + 1];
  std::vector<float> inv_var, wfwd, wadj;   // 1/sigma^2; padded PSF weight rows (forward, adjoint)
  std::vector<float> wsep;                  // rank-one factors [4][KP] (see SysDev::psf_sep)
  bool rank1 = false;
};
int ensure_constants(int device);
bool valid_geometry(const rtu_geometry* g);
void fill_geometry(const rtu_geometry* g, SysDev& h);
size_t carve_workspace(SysDev& h, int B, char* base);
size_t carve_observation(SysDev& h, int B, int M, char* base);
size_t carve_fit(FitDev& F, int S, int max_steps, char* base);
void prepare_observation(const rtu_geometry* g, const float* noise_sigma, const float* psf,
                         const uint8_t* arc_mask, ObsHost& o);
hipError_t upload_observation(const SysDev& h, const float* image, const float* psf, const uint8_t* arc_mask,
                              const ObsHost& o, hipStream_t s);
double elbo_constant(const std::vector<float>& inv_var, int n_src2, int dim);
hipError_t init_fit_state(const FitDev& F, const float* mu0, const float* rho0, int n_sub, hipStream_t s);

// LDS sizing shared by both launch paths
size_t ray_lds_bytes(const SysDev& h, bool adjoint, bool lds_grid);
int adj_window_cap(const SysDev& h);
bool adj_lds_grid(const SysDev& h);
size_t psf_lds_bytes(int KP);
int fft_lds_cap(int n_src);          // float2 slots of the FFT line buffer for this grid
size_t gp_lds_bytes(int n_src);      // dynamic LDS of a split GP line pass
size_t prep_lds_bytes(int n_src);
size_t post_lds_bytes(int n_src, int n_lens);

// shared launches over many systems (serving): one work item per task
struct FleetLaunch {
  const SysDev* sys;          // device [n_slots]
  const FitDev* fit;          // device [n_slots]
  const Task *t_prep, *t_psf, *t_post, *t_param, *t_sample, *t_fit, *t_gp;
  int n_prep, n_psf, n_post, n_param, n_sample, n_fit, n_gp;   // t_gp: split GP line groups
  const Task* t_mr;           // masked-ray chunks (systems with mr_nchunk > 0)
  int n_mr;
  // forward ray tiles by main deflector: [0] SIE, [1] EPL
  const Task* t_fwd[2];
  int n_fwd[2];
  // adjoint ray tiles by LDS mode ([0] d loss / d s in LDS, [1] in global
  // memory), then by main deflector
  const Task* t_adj[2][2];
  int n_adj[2][2];
  int adj_sub[2][2];          // the list has a system with subhaloes
  size_t lds_rays_fwd, lds_rays_adj, lds_psf, lds_prep, lds_post, lds_gp;
  int adam_threads;           // ADAM_P x the sample groups of the largest sample count (<= ADAM_THREADS)
  int prep_threads;           // prep workgroup size for the largest mask (prep_threads)
};
// One stage (RTU_STAGE_*) of a shared launch; eps (device [S][dim] per fit,
// only for a single-fit table) replaces the Philox draws when not null.
hipError_t launch_fleet_stage(const FleetLaunch& L, int stage, int round, const float* eps, hipStream_t s);

// Device copies of the descriptors and work lists of a set of systems/fits.
struct DeviceTables {
  SysDev* d_sys = nullptr;
  FitDev* d_fit = nullptr;
  Task* d_tasks = nullptr;
  size_t cap_slots = 0, cap_tasks = 0;
  // synchronous upload; the previous tables must no longer be in use
  int upload(const std::vector<SysDev>& sys, const std::vector<FitDev>& fit, FleetLaunch& L);
  void release();
};

}  // namespace rtu
