// Runs one evaluation (forward and gradient) of an input file through the
// library's C ABI on the host emulation of the device, and writes every
// output: loss[B], chi2_mask[B] (double), status[B] (uint32), grad_lens[B][nl],
// grad_ps[B][4], grad_latent[B][n][n], model[B][N][N] (float).
//   driver <inputs> <outputs> <mode: 0 plan, 1 allocation-free> <geometry flags>
// (header word 8 = 1: per-pixel ray weights follow the inputs), then (plan
// mode, zeros otherwise) the selected rays [B][2][2K] and the standardisation
// [B][3] of RTU_DBG_SELECT and RTU_DBG_STD.
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "hip/hip_runtime.h"
#include "rtu.h"

template <class T>
static T* dev(const std::vector<T>& h) {
  T* d;
  hipMalloc(&d, h.size() * sizeof(T));
  hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
  return d;
}
template <class T>
static T* dev_empty(size_t n) {
  T* d;
  hipMalloc(&d, n * sizeof(T));
  return d;
}

int main(int argc, char** argv) {
  if (argc < 5) return 64;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 65;
  int hi[9];
  float hf[2];
  if (fread(hi, 4, 9, f) != 9 || fread(hf, 4, 2, f) != 2) return 66;
  const int N = hi[0], ss = hi[1], n = hi[2], KP = hi[3], nsm = hi[4], ng = hi[5], B = hi[6], nl = hi[7];
  auto rd = [&](auto& v, size_t cnt) {
    v.resize(cnt);
    if (fread(v.data(), sizeof(v[0]), cnt, f) != cnt) exit(67);
  };
  std::vector<float> image, sigma, psf, lens, ps, lat;
  std::vector<uint8_t> mask;
  std::vector<int> nsub;
  rd(image, (size_t)N * N); rd(sigma, (size_t)N * N); rd(psf, (size_t)KP * KP); rd(mask, (size_t)N * N);
  rd(lens, (size_t)B * nl); rd(ps, (size_t)B * 4); rd(lat, (size_t)B * n * n); rd(nsub, (size_t)B);
  std::vector<float> wts;
  if (hi[8] == 1) rd(wts, (size_t)N * N);     // ray weights of the weighted grid
  fclose(f);
  const int mode = atoi(argv[3]);
  const unsigned flags = (unsigned)atoi(argv[4]);
  rtu_geometry g{N, ss, n, KP, nsm, RTU_K_NODES, hf[0], hf[1], flags, ng};
  double* loss = dev_empty<double>(B);
  double* c2m = dev_empty<double>(B);
  uint32_t* st = dev_empty<uint32_t>(B);
  float* gl = dev_empty<float>((size_t)B * nl);
  float* gp = dev_empty<float>((size_t)B * 4);
  float* gw = dev_empty<float>((size_t)B * n * n);
  float* model = dev_empty<float>((size_t)B * N * N);
  float* dl = dev(lens);
  float* dp = dev(ps);
  float* dw = dev(lat);
  int* dn = dev(nsub);
  int rc;
  // plan mode: the selected rays and the standardisation of every sample too
  std::vector<int> sel((size_t)B * 4 * RTU_K_NODES, 0);
  std::vector<double> sd((size_t)B * 3, 0.0);
  if (mode == 0) {
    rtu_plan p;
    if ((rc = rtu_plan_create(&g, B, 0, &p))) return 70;
    if ((rc = rtu_set_observation(p, image.data(), sigma.data(), psf.data(), mask.data(), nullptr))) return 71;
    if (!wts.empty() && (rc = rtu_set_ray_weights(p, wts.data(), nullptr))) return 74;
    if ((rc = rtu_loss_grad(p, B, dl, dn, dp, dw, loss, c2m, gl, gp, gw, model, st, nullptr))) return 72;
    for (int b = 0; b < B; ++b) {
      if (rtu_debug_fetch(p, RTU_DBG_SELECT, b, sel.data() + (size_t)b * 4 * RTU_K_NODES,
                          4 * RTU_K_NODES * sizeof(int), nullptr) ||
          rtu_debug_fetch(p, RTU_DBG_STD, b, sd.data() + (size_t)b * 3, 3 * sizeof(double), nullptr))
        return 75;
    }
    rtu_plan_destroy(p);
  } else {
    float* di = dev(image);
    float* ds = dev(sigma);
    float* dk = dev(psf);
    uint8_t* dm = dev(mask);
    if ((rc = rtu_loss_grad_noalloc(&g, B, di, ds, dk, dm, dl, dn, dp, dw, loss, c2m, gl, gp, gw, model, st,
                                    nullptr)))
      return 73;
  }
  FILE* o = fopen(argv[2], "wb");
  fwrite(loss, 8, B, o);
  fwrite(c2m, 8, B, o);
  fwrite(st, 4, B, o);
  fwrite(gl, 4, (size_t)B * nl, o);
  fwrite(gp, 4, (size_t)B * 4, o);
  fwrite(gw, 4, (size_t)B * n * n, o);
  fwrite(model, 4, (size_t)B * N * N, o);
  fwrite(sel.data(), 4, sel.size(), o);
  fwrite(sd.data(), 8, sd.size(), o);
  fclose(o);
  return 0;
}
