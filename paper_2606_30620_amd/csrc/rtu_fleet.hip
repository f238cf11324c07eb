// Serving fleet: many variational fits of different lens systems advanced
// together, one ELBO + Adam step per round, in shared kernel launches.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

#include "rtu_internal.h"

using namespace rtu;

namespace {

// First-fit allocator over the arena [0, size) with 256-byte granules.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t& off) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

struct Entry {
  int64_t ticket = 0;
  rtu_geometry g;
  int S = 0, steps = 0, n_sub = 0;
  float lr = 0.f;
  uint64_t seed = 0;
  uint32_t log_mask[RTU_LOG_MASK_WORDS] = {0, 0, 0};
  std::vector<float> image, sigma, psf, mu0, rho0;
  std::vector<uint8_t> mask;
  ObsHost obs;
  size_t bytes = 0, off = 0;
  SysDev h;
  FitDev F;
  int round0 = 0;
};

struct Result {
  std::vector<float> mu, rho;
  std::vector<double> trace;
  uint32_t status = 0;
};

// Layout of one admitted fit inside its arena block: observation and
// mask-dependent buffers, evaluation workspace for S samples, fit state.
size_t layout(Entry& e, char* base) {
  fill_geometry(&e.g, e.h);
  const int M = (int)e.obs.idx.size();
  size_t off = carve_observation(e.h, e.S, M, base);
  off = (off + 255) & ~(size_t)255;
  off += carve_workspace(e.h, e.S, base ? base + off : nullptr);
  off = (off + 255) & ~(size_t)255;
  FitDev& F = e.F;
  memset(&F, 0, sizeof(F));
  F.S = e.S;
  F.n_lens = e.h.n_lens;
  F.n_src2 = e.h.n_src * e.h.n_src;
  F.dim = F.n_lens + 4 + F.n_src2;
  off += carve_fit(F, e.S, e.steps, base ? base + off : nullptr);
  e.h.M = M;
  return off + 256;
}

bool valid_request(const rtu_fit_request* r) {
  return r && valid_geometry(&r->geom) && r->image && r->noise_sigma && r->psf && r->arc_mask && r->mu0 &&
         r->rho0 && r->samples >= 1 && r->steps >= 1 && r->n_sub >= 0 && r->n_sub <= r->geom.n_sub_max;
}

}  // namespace

namespace rtu {

int DeviceTables::upload(const std::vector<SysDev>& sys, const std::vector<FitDev>& fit, FleetLaunch& L) {
  const size_t n = sys.size();
  std::vector<Task> prep, psf, post, param, samp, fits, gp, mr, fwd[2], adj[2][2];
  int adj_sub[2][2] = {{0, 0}, {0, 0}};
  size_t lds_f = 0, lds_a = 0, lds_p = 0, lds_pr = 0, lds_po = 0, lds_g = 0;
  for (size_t i = 0; i < n; ++i) {
    const SysDev& h = sys[i];
    const FitDev& F = fit[i];
    const int si = (int)i, S = h.batch;
    if (h.n_sub_max > 0) adj_sub[h.lds_adj ? 0 : 1][h.epl ? 1 : 0] = 1;
    for (int b = 0; b < S; ++b) {
      for (int c = 0; c < h.mr_nchunk; ++c) mr.push_back(make_int4(si, b, c, 0));
      for (int r = 0; r < 3; ++r) prep.push_back(make_int4(si, b, r, 0));
      if (gp_split(h.n_src))
        for (int g = 0; g < h.n_src / GP_LINES; ++g) gp.push_back(make_int4(si, b, g, 0));
      for (int t = 0; t < h.ray_tiles; ++t) {
        fwd[h.epl ? 1 : 0].push_back(make_int4(si, b, t, 0));
        adj[h.lds_adj ? 0 : 1][h.epl ? 1 : 0].push_back(make_int4(si, b, t, 0));
      }
      for (int t = 0; t < h.psf_tiles; ++t) psf.push_back(make_int4(si, b, t, 0));
      for (int r = 0; r < (h.want_grad ? 2 : 1); ++r) post.push_back(make_int4(si, b, r, 0));
    }
    const int nblk = (F.dim + 255) / 256;
    for (int j = 0; j < (F.dim + ADAM_P - 1) / ADAM_P; ++j) param.push_back(make_int4(si, j, 0, 0));
    for (int j = 0; j < nblk; ++j) {
      for (int s = 0; s < S; ++s) samp.push_back(make_int4(si, j, s, 0));
    }
    fits.push_back(make_int4(si, 0, 0, 0));
    lds_f = std::max(lds_f, ray_lds_bytes(h, false, false));
    lds_a = std::max(lds_a, ray_lds_bytes(h, true, h.lds_adj != 0));
    lds_p = std::max(lds_p, psf_lds_bytes(h.psf_k));
    lds_pr = std::max(lds_pr, prep_lds_bytes(h.n_src));
    lds_po = std::max(lds_po, post_lds_bytes(h.n_src, h.n_lens));
    if (gp_split(h.n_src)) lds_g = std::max(lds_g, gp_lds_bytes(h.n_src));
  }
  std::vector<Task> all;
  size_t off[14];
  std::vector<Task>* lists[14] = {&prep, &psf, &post, &param, &samp, &fits, &fwd[0], &fwd[1],
                                  &adj[0][0], &adj[0][1], &adj[1][0], &adj[1][1], &gp, &mr};
  for (int k = 0; k < 14; ++k) {
    off[k] = all.size();
    all.insert(all.end(), lists[k]->begin(), lists[k]->end());
  }
  if (n > cap_slots) {
    if (d_sys) (void)hipFree(d_sys);
    if (d_fit) (void)hipFree(d_fit);
    d_sys = nullptr;
    d_fit = nullptr;
    cap_slots = std::max(n, (size_t)8) * 2;
    if (hipMalloc(&d_sys, cap_slots * sizeof(SysDev)) != hipSuccess) return RTU_ENOMEM;
    if (hipMalloc(&d_fit, cap_slots * sizeof(FitDev)) != hipSuccess) return RTU_ENOMEM;
  }
  if (all.size() > cap_tasks) {
    if (d_tasks) (void)hipFree(d_tasks);
    d_tasks = nullptr;
    cap_tasks = std::max(all.size(), (size_t)256) * 2;
    if (hipMalloc(&d_tasks, cap_tasks * sizeof(Task)) != hipSuccess) return RTU_ENOMEM;
  }
  if (n && (hipMemcpy(d_sys, sys.data(), n * sizeof(SysDev), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_fit, fit.data(), n * sizeof(FitDev), hipMemcpyHostToDevice) != hipSuccess))
    return RTU_EHIP;
  if (!all.empty() && hipMemcpy(d_tasks, all.data(), all.size() * sizeof(Task), hipMemcpyHostToDevice) != hipSuccess)
    return RTU_EHIP;
  L.sys = d_sys;
  L.fit = d_fit;
  L.t_prep = d_tasks + off[0];  L.n_prep = (int)prep.size();
  L.t_psf = d_tasks + off[1];   L.n_psf = (int)psf.size();
  L.t_post = d_tasks + off[2];  L.n_post = (int)post.size();
  L.t_param = d_tasks + off[3]; L.n_param = (int)param.size();
  L.t_sample = d_tasks + off[4]; L.n_sample = (int)samp.size();
  L.t_fit = d_tasks + off[5];   L.n_fit = (int)fits.size();
  L.t_gp = d_tasks + off[12];   L.n_gp = (int)gp.size();
  L.t_mr = d_tasks + off[13];   L.n_mr = (int)mr.size();
  {
    int smax = 1, g = 1;
    for (size_t i = 0; i < n; ++i) smax = std::max(smax, fit[i].S);
    while (g < smax && ADAM_P * g < ADAM_THREADS) g *= 2;
    L.adam_threads = ADAM_P * g;
    L.prep_threads = PREP_THREADS;
    for (size_t i = 0; i < n; ++i)
      L.prep_threads = std::max(L.prep_threads, prep_threads(sys[i].obs_dyn ? 0 : sys[i].M, sys[i].n_src));
  }
  L.lds_gp = lds_g;
  for (int k = 0; k < 2; ++k) {
    L.t_fwd[k] = d_tasks + off[6 + k]; L.n_fwd[k] = (int)fwd[k].size();
    for (int e = 0; e < 2; ++e) {
      L.t_adj[k][e] = d_tasks + off[8 + 2 * k + e];
      L.n_adj[k][e] = (int)adj[k][e].size();
      L.adj_sub[k][e] = adj_sub[k][e];
    }
  }
  L.lds_rays_fwd = lds_f;
  L.lds_rays_adj = lds_a;
  L.lds_psf = lds_p;
  L.lds_prep = lds_pr;
  L.lds_post = lds_po;
  return RTU_OK;
}

void DeviceTables::release() {
  if (d_sys) (void)hipFree(d_sys);
  if (d_fit) (void)hipFree(d_fit);
  if (d_tasks) (void)hipFree(d_tasks);
  d_sys = nullptr;
  d_fit = nullptr;
  d_tasks = nullptr;
  cap_slots = cap_tasks = 0;
}

}  // namespace rtu

// Pinned host staging for the copies of a sync point (admitted fits'
// observation tables and initial guide, retired fits' results): blocks of
// 16 MiB, at most 64 MiB in all, handed out in order; a request larger than
// a block gets a block of its own whatever the total.  take() returns null
// when the pool is full: the caller then synchronises the stream (every copy
// out of or into the pool has completed) and resets it.  Each sync point
// starts from a reset pool.
struct Staging {
  static constexpr size_t BLOCK = (size_t)16 << 20, CAP = (size_t)64 << 20;
  std::vector<std::pair<char*, size_t>> blocks;
  size_t cur = 0, used = 0, total = 0;
  char* take(size_t bytes) {
    used = (used + 255) & ~(size_t)255;
    while (cur < blocks.size() && used + bytes > blocks[cur].second) { ++cur; used = 0; }
    if (cur == blocks.size()) {
      const size_t cap = std::max(bytes, BLOCK);
      char* p = nullptr;
      if ((!blocks.empty() && bytes <= BLOCK && total + cap > CAP) ||
          hipHostMalloc(reinterpret_cast<void**>(&p), cap, hipHostMallocDefault) != hipSuccess)
        return nullptr;
      blocks.push_back({p, cap});
      total += cap;
      used = 0;
    }
    char* p = blocks[cur].first + used;
    used += bytes;
    return p;
  }
  void reset() { cur = 0; used = 0; }
  void release() {
    for (auto& b : blocks) (void)hipHostFree(b.first);
    blocks.clear();
    total = 0;
    reset();
  }
};

struct rtu_fleet_s {
  int device = 0;
  size_t budget = 0;
  int max_fits = 0, sync_every = 1;
  char* arena = nullptr;
  Arena alloc;
  std::deque<Entry> queue;
  std::vector<Entry> active;
  std::deque<int64_t> done;
  std::unordered_map<int64_t, Result> results;
  int64_t next_ticket = 1;
  int round = 0, since_sync = 0;
  int64_t rounds_run = 0;
  DeviceTables tables;
  FleetLaunch L{};
  bool dirty = true;
  Staging stage;
};

namespace {

int upload_tables(rtu_fleet f) {
  std::vector<SysDev> sys;
  std::vector<FitDev> fit;
  for (const Entry& e : f->active) {
    sys.push_back(e.h);
    fit.push_back(e.F);
  }
  const int rc = f->tables.upload(sys, fit, f->L);
  if (rc == RTU_OK) f->dirty = false;
  return rc;
}

bool finished(const rtu_fleet f, const Entry& e) { return f->round - e.round0 >= e.steps; }

int admit_one(rtu_fleet f, hipStream_t s) {
  Entry& q = f->queue.front();
  size_t off;
  if (!f->alloc.alloc(q.bytes, off)) return 0;
  Entry e = std::move(q);
  f->queue.pop_front();
  e.off = off;
  char* base = f->arena + off;
  layout(e, base);
  SysDev& h = e.h;
  FitDev& F = e.F;
  h.batch = e.S;
  h.want_grad = 1;
  h.lens = F.z_lens; h.n_sub = F.n_sub; h.ps = F.z_ps; h.latent = F.z_lat;
  h.loss = F.loss; h.chi2m = F.chi2m; h.g_lens = F.g_lens; h.g_ps = F.g_ps; h.g_lat = F.g_lat;
  h.model = nullptr; h.status = F.status;
  h.lds_adj = adj_lds_grid(h) ? 1 : 0;
  h.psf_rank1 = e.obs.rank1 ? 1 : 0;
  e.round0 = f->round;
  h.round0 = f->round;
  h.nsteps = e.steps;
  F.round0 = f->round;
  F.nsteps = e.steps;
  F.lr = e.lr;
  F.seed_lo = (uint32_t)e.seed;
  F.seed_hi = (uint32_t)(e.seed >> 32);
  for (int w = 0; w < RTU_LOG_MASK_WORDS; ++w) F.log_mask[w] = e.log_mask[w];
  F.elbo_const = elbo_constant(e.obs.inv_var, F.n_src2, F.dim);
  // the observation region (carved first, from base, up to zbuf) and the
  // initial fit state, staged in pinned memory laid out as on the device and
  // sent in four asynchronous copies
  {
    const int M = (int)e.obs.idx.size();
    const size_t ob = (size_t)(reinterpret_cast<const char*>(h.zbuf) - base);
    const size_t fb = (size_t)(reinterpret_cast<const char*>(F.rho + F.dim) - reinterpret_cast<const char*>(F.mu));
    // a full pool: the copies issued from it complete, then it is reused
    auto stage = [&](size_t bytes) -> char* {
      char* p = f->stage.take(bytes);
      if (!p && hipStreamSynchronize(s) == hipSuccess) {
        f->stage.reset();
        p = f->stage.take(bytes);
      }
      return p;
    };
    char* so = stage(ob);
    if (!so) return -1;
    SysDev hs = h;
    carve_observation(hs, e.S, M, so);
    const size_t N2 = (size_t)h.n_img * h.n_img, kw = (size_t)h.psf_k * psf_ws(h.psf_k);
    memcpy(const_cast<float*>(hs.image), e.image.data(), N2 * 4);
    memcpy(const_cast<float*>(hs.inv_var), e.obs.inv_var.data(), N2 * 4);
    memcpy(const_cast<float*>(hs.psf_flip), e.obs.wfwd.data(), kw * 4);
    memcpy(const_cast<float*>(hs.psf), e.obs.wadj.data(), kw * 4);
    memcpy(const_cast<float*>(hs.psf_sep), e.obs.wsep.data(), e.obs.wsep.size() * 4);
    memcpy(const_cast<uint8_t*>(hs.mask), e.mask.data(), N2);
    if (M) memcpy(const_cast<int*>(hs.mask_idx), e.obs.idx.data(), (size_t)M * 4);
    if (M) memcpy(const_cast<float2*>(hs.mask_xy), e.obs.xy.data(), (size_t)M * sizeof(float2));
    memcpy(const_cast<int*>(hs.rank_j), e.obs.rank_j, sizeof(e.obs.rank_j));
    memcpy(const_cast<double*>(hs.rank_t), e.obs.rank_t, sizeof(e.obs.rank_t));
    memcpy(const_cast<int*>(hs.tsel), e.obs.tsel, sizeof(e.obs.tsel));
    if (hipMemcpyAsync(base, so, ob, hipMemcpyHostToDevice, s) != hipSuccess) return -1;
    // mu and rho are carved one after the other, then the four Adam moments
    // (zeroed on the device)
    const size_t fb2 = (fb + 255) & ~(size_t)255;
    char* sf = stage(fb2 + (size_t)F.S * 4 + 4);
    if (!sf) return -1;
    int* sn = reinterpret_cast<int*>(sf + fb2);
    memcpy(sf, e.mu0.data(), (size_t)F.dim * 4);
    memcpy(sf + (reinterpret_cast<const char*>(F.rho) - reinterpret_cast<const char*>(F.mu)), e.rho0.data(),
           (size_t)F.dim * 4);
    for (int q = 0; q < F.S; ++q) sn[q] = e.n_sub;
    sn[F.S] = 0;
    const size_t zb = (size_t)(reinterpret_cast<const char*>(F.v_rho + F.dim) - reinterpret_cast<const char*>(F.m_mu));
    if (hipMemcpyAsync(F.mu, sf, fb, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(F.m_mu, 0, zb, s) != hipSuccess ||
        hipMemcpyAsync(F.n_sub, sn, (size_t)F.S * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(F.status_acc, sn + F.S, 4, hipMemcpyHostToDevice, s) != hipSuccess)
      return -1;
  }
  // the host copies are no longer needed once on the device
  e.image.clear(); e.image.shrink_to_fit();
  e.sigma.clear(); e.sigma.shrink_to_fit();
  e.mask.clear(); e.mask.shrink_to_fit();
  f->active.push_back(std::move(e));
  return 1;
}

int sync_point(rtu_fleet f, hipStream_t s) {
  if (hipStreamSynchronize(s) != hipSuccess) return RTU_EHIP;
  f->stage.reset();   // every copy of the previous sync point has completed
  // retire: each finished fit's guide, ELBO trace and status into pinned
  // staging (asynchronous copies), one synchronisation for all of them
  std::vector<Entry> keep, gone;
  std::vector<char*> at;
  bool changed = false;
  // the staged results so far: wait for their copies, read them, reuse the pool
  auto drain = [&]() -> int {
    if (gone.empty()) return RTU_OK;
    if (hipStreamSynchronize(s) != hipSuccess) return RTU_EHIP;
    for (size_t i = 0; i < gone.size(); ++i) {
      const Entry& e = gone[i];
      const char* p = at[i];
      const size_t d4 = (size_t)e.F.dim * 4;
      Result r;
      r.mu.resize(e.F.dim);
      r.rho.resize(e.F.dim);
      r.trace.resize(e.steps);
      memcpy(r.mu.data(), p, d4);
      memcpy(r.rho.data(), p + d4, d4);
      memcpy(r.trace.data(), p + 2 * d4, (size_t)e.steps * 8);
      memcpy(&r.status, p + 2 * d4 + (size_t)e.steps * 8, 4);
      f->alloc.release(e.off, e.bytes);
      f->results[e.ticket] = std::move(r);
      f->done.push_back(e.ticket);
    }
    gone.clear();
    at.clear();
    f->stage.reset();
    changed = true;
    return RTU_OK;
  };
  for (Entry& e : f->active) {
    if (!finished(f, e)) {
      keep.push_back(std::move(e));
      continue;
    }
    const size_t d4 = (size_t)e.F.dim * 4, bytes = 2 * d4 + (size_t)e.steps * 8 + 8;
    char* p = f->stage.take(bytes);
    if (!p) {
      const int rc = drain();
      if (rc) return rc;
      p = f->stage.take(bytes);
      if (!p) return RTU_ENOMEM;
    }
    if (hipMemcpyAsync(p, e.F.mu, d4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(p + d4, e.F.rho, d4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(p + 2 * d4, e.F.trace, (size_t)e.steps * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(p + 2 * d4 + (size_t)e.steps * 8, e.F.status_acc, 4, hipMemcpyDeviceToHost, s) != hipSuccess)
      return RTU_EHIP;
    at.push_back(p);
    gone.push_back(std::move(e));
  }
  {
    const int rc = drain();   // also resets the pool for the admissions below
    if (rc) return rc;
  }
  f->active = std::move(keep);
  // admit, first come first served
  while (!f->queue.empty() && (int)f->active.size() < f->max_fits) {
    const int rc = admit_one(f, s);
    if (rc < 0) return RTU_EHIP;
    if (rc == 0) break;
    changed = true;
  }
  if (changed) f->dirty = true;
  f->since_sync = 0;
  return RTU_OK;
}

}  // namespace

extern "C" {

size_t rtu_fleet_request_bytes(const rtu_fit_request* r) {
  if (!valid_request(r)) return 0;
  Entry e;
  e.g = r->geom;
  e.S = r->samples;
  e.steps = r->steps;
  const size_t N2 = (size_t)r->geom.n_img * r->geom.n_img;
  e.obs.idx.resize(std::count_if(r->arc_mask, r->arc_mask + N2, [](uint8_t v) { return v != 0; }));
  return layout(e, nullptr);
}

int rtu_fleet_create(int32_t device, size_t hbm_budget, int32_t max_fits, int32_t sync_every, rtu_fleet* out) {
  if (!out || hbm_budget < 4096 || max_fits < 1 || sync_every < 1) return RTU_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return RTU_EINVAL;
  int rc = ensure_constants(device);
  if (rc) return rc;
  rtu_fleet f = new rtu_fleet_s();
  f->device = device;
  f->budget = hbm_budget;
  f->max_fits = max_fits;
  f->sync_every = sync_every;
  if (hipMalloc(&f->arena, hbm_budget) != hipSuccess) {
    delete f;
    return RTU_ENOMEM;
  }
  f->alloc.reset(hbm_budget);
  *out = f;
  return RTU_OK;
}

int rtu_fleet_destroy(rtu_fleet f) {
  if (!f) return RTU_EINVAL;
  (void)hipSetDevice(f->device);
  (void)hipDeviceSynchronize();
  if (f->arena) (void)hipFree(f->arena);
  f->tables.release();
  f->stage.release();
  delete f;
  return RTU_OK;
}

int rtu_fleet_submit(rtu_fleet f, const rtu_fit_request* r, int64_t* ticket) {
  if (!f || !ticket || !valid_request(r)) return RTU_EINVAL;
  Entry e;
  e.g = r->geom;
  e.S = r->samples;
  e.steps = r->steps;
  e.n_sub = r->n_sub;
  e.lr = r->lr;
  e.seed = r->seed;
  for (int w = 0; w < RTU_LOG_MASK_WORDS; ++w) e.log_mask[w] = r->log_mask[w];
  const size_t N2 = (size_t)r->geom.n_img * r->geom.n_img, K2 = (size_t)r->geom.psf_size * r->geom.psf_size;
  SysDev tmp;
  fill_geometry(&r->geom, tmp);
  const size_t dim = (size_t)tmp.n_lens + 4 + (size_t)tmp.n_src * tmp.n_src;
  e.image.assign(r->image, r->image + N2);
  e.sigma.assign(r->noise_sigma, r->noise_sigma + N2);
  e.psf.assign(r->psf, r->psf + K2);
  e.mask.assign(r->arc_mask, r->arc_mask + N2);
  e.mu0.assign(r->mu0, r->mu0 + dim);
  e.rho0.assign(r->rho0, r->rho0 + dim);
  prepare_observation(&e.g, e.sigma.data(), e.psf.data(), e.mask.data(), e.obs);
  e.bytes = layout(e, nullptr);
  if (e.bytes > f->budget) return RTU_ENOMEM;
  e.ticket = f->next_ticket++;
  *ticket = e.ticket;
  f->queue.push_back(std::move(e));
  return RTU_OK;
}

int rtu_fleet_sync(rtu_fleet f, void* stream) {
  if (!f) return RTU_EINVAL;
  if (hipSetDevice(f->device) != hipSuccess) return RTU_EHIP;
  return sync_point(f, reinterpret_cast<hipStream_t>(stream));
}

int rtu_fleet_run(rtu_fleet f, int32_t rounds, void* stream) {
  if (!f || rounds < 0) return RTU_EINVAL;
  if (hipSetDevice(f->device) != hipSuccess) return RTU_EHIP;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int r = 0; r < rounds; ++r) {
    int running = 0, done = 0;
    for (const Entry& e : f->active) (finished(f, e) ? done : running)++;
    const bool can_admit = !f->queue.empty() && (int)f->active.size() < f->max_fits;
    if ((done || can_admit) && (f->since_sync >= f->sync_every || running == 0)) {
      int rc = sync_point(f, s);
      if (rc) return rc;
      running = 0;
      for (const Entry& e : f->active) running += !finished(f, e);
    }
    if (running == 0) break;
    // new tables (fits admitted or retired): the sampling launch draws the
    // first samples of the new fits (and again, identically, those of the
    // others); otherwise every fit's samples come from its last Adam update
    bool fresh = false;
    if (f->dirty) {
      int rc = upload_tables(f);
      if (rc) return rc;
      fresh = true;
    }
    const int order[] = {RTU_STAGE_SAMPLE, RTU_STAGE_PREP, RTU_STAGE_RAYS_FWD, RTU_STAGE_PSF_FWD,
                         RTU_STAGE_PSF_ADJ, RTU_STAGE_RAYS_ADJ, RTU_STAGE_POST, RTU_STAGE_ADAM};
    for (int st : order) {
      if (st == RTU_STAGE_SAMPLE && !fresh) continue;
      if (launch_fleet_stage(f->L, st, f->round, nullptr, s) != hipSuccess) return RTU_EHIP;
    }
    f->round++;
    f->since_sync++;
    f->rounds_run++;
  }
  return RTU_OK;
}

int rtu_fleet_poll(rtu_fleet f, int64_t* tickets, int32_t max, int32_t* n) {
  if (!f || !n || (max > 0 && !tickets)) return RTU_EINVAL;
  int k = 0;
  while (k < max && !f->done.empty()) {
    tickets[k++] = f->done.front();
    f->done.pop_front();
  }
  *n = k;
  return RTU_OK;
}

int rtu_fleet_result(rtu_fleet f, int64_t ticket, float* mu, float* rho, double* elbo, int32_t max_trace,
                     int32_t* n_trace, uint32_t* status) {
  if (!f) return RTU_EINVAL;
  auto it = f->results.find(ticket);
  if (it == f->results.end()) return RTU_ENOTFOUND;
  const Result& r = it->second;
  if (mu) memcpy(mu, r.mu.data(), r.mu.size() * 4);
  if (rho) memcpy(rho, r.rho.data(), r.rho.size() * 4);
  if (elbo && max_trace > 0)
    memcpy(elbo, r.trace.data(), std::min((size_t)max_trace, r.trace.size()) * 8);
  if (n_trace) *n_trace = (int32_t)r.trace.size();
  if (status) *status = r.status;
  f->results.erase(it);
  return RTU_OK;
}

int rtu_fleet_stats(rtu_fleet f, int32_t* active, int32_t* queued, size_t* bytes_in_use, int64_t* rounds) {
  if (!f) return RTU_EINVAL;
  if (active) *active = (int32_t)f->active.size();
  if (queued) *queued = (int32_t)f->queue.size();
  if (bytes_in_use) *bytes_in_use = f->alloc.used();
  if (rounds) *rounds = f->rounds_run;
  return RTU_OK;
}

}  // extern "C"
