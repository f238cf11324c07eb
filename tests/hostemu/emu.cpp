// Host emulation of the device runtime for the bounds-checking build: kernel
// launches (every workgroup of a grid in turn, its lanes as threads) and
// allocations followed by poisoned red zones.
#include "hip/hip_runtime.h"

thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
thread_local EmuBlock* emu_blk;
std::mutex emu_atomic_mu;

static size_t rz_of(size_t n) { size_t r = n < 4096 ? 4096 : n; return (r + 255) & ~(size_t)255; }
static std::mutex g_mu;
static std::vector<std::pair<void*, size_t>> g_allocs;

hipError_t hipMalloc(void** p, size_t n) {
  const size_t a = (n + 255) & ~(size_t)255, tot = a + rz_of(n);
  char* b = (char*)aligned_alloc(256, tot);
  if (!b) return hipErrorUnknown;
  memset(b, 0xA5, tot);                       // device memory starts with garbage
  ASAN_POISON_MEMORY_REGION(b + n, tot - n);
  std::lock_guard<std::mutex> g(g_mu);
  g_allocs.push_back({b, tot});
  *p = b;
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, int) { return hipMalloc(p, n); }
hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  std::lock_guard<std::mutex> g(g_mu);
  for (auto it = g_allocs.begin(); it != g_allocs.end(); ++it)
    if (it->first == p) {
      ASAN_UNPOISON_MEMORY_REGION(p, it->second);
      free(p);
      g_allocs.erase(it);
      return hipSuccess;
    }
  fprintf(stderr, "emu: hipFree of unknown pointer %p\n", p);
  abort();
}
hipError_t hipHostFree(void* p) { return hipFree(p); }

// Carve guard: the buffer [p, p+n) becomes addressable, the alignment slack
// and a red zone as large as the buffer after it are poisoned.
size_t emu_guard(char* base, char* p, size_t n, size_t off) {
  const size_t aligned = (off + 255) & ~(size_t)255, rz = rz_of(n);
  if (base) {
    ASAN_UNPOISON_MEMORY_REGION(p, n);
    ASAN_POISON_MEMORY_REGION(base + off, aligned - off + rz);
  }
  return aligned + rz;
}

__attribute__((no_sanitize("address"))) void emu_copy(void* d, const void* s, size_t n) {
  volatile char* dd = (volatile char*)d;
  const volatile char* ss = (const volatile char*)s;
  if (dd < ss) for (size_t i = 0; i < n; ++i) dd[i] = ss[i];
  else for (size_t i = n; i-- > 0;) dd[i] = ss[i];
}

void emu_run_grid(dim3 g, dim3 b, size_t lds, const char* name, const std::function<void()>& body) {
  const unsigned nt = b.x;
  if (b.y != 1 || b.z != 1 || nt % 64) { fprintf(stderr, "emu: block shape\n"); abort(); }
  if (getenv("EMU_VERBOSE")) fprintf(stderr, "emu: %s grid (%u,%u,%u) block %u lds %zu\n", name, g.x, g.y, g.z, nt, lds);
  for (unsigned bz = 0; bz < g.z; ++bz)
    for (unsigned by = 0; by < g.y; ++by)
      for (unsigned bx = 0; bx < g.x; ++bx) {
        std::barrier<> bar(nt);
        std::vector<EmuWave> waves(nt / 64);
        std::vector<std::barrier<>*> wb;
        for (auto& w : waves) { w.bar = new std::barrier<>(64); wb.push_back(w.bar); }
        EmuBlock blk{&bar, waves.data(), (unsigned char*)malloc(lds ? lds : 1)};
        memset(blk.dyn, 0xC3, lds ? lds : 1);     // LDS starts with garbage
        std::vector<std::thread> th;
        th.reserve(nt);
        for (unsigned t = 0; t < nt; ++t)
          th.emplace_back([&, t]() {
            threadIdx = dim3(t, 0, 0);
            blockIdx = dim3(bx, by, bz);
            blockDim = dim3(nt, 1, 1);
            gridDim = g;
            emu_blk = &blk;
            body();
            blk.waves[t >> 6].bar->arrive_and_drop();
            bar.arrive_and_drop();
          });
        for (auto& x : th) x.join();
        free(blk.dyn);
        for (auto* p : wb) delete p;
      }
}
