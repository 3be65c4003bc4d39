// Runtime of the multilevel GDSW library: hierarchy construction (section 2.1
// per level, recursion of section 2.2), the apply of eq. (2.2) and restarted
// FGMRES (section 3), behind the C ABI declared in include/gdsw.h.
#include "../../include/gdsw.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "maps.h"

namespace gdsw {

namespace {

thread_local std::string g_last_error;

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Wait for an event by polling it: the Krylov loop waits once per iteration for
// a few microseconds of copy after its apply, so a blocking synchronization's
// wake-up latency is avoided; after the first 50 us the thread yields its core
// between queries, so that concurrent solves on other threads (serving) are
// not starved by spinning ones.
void wait_event_polling(hipEvent_t e) {
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t q;
  while ((q = hipEventQuery(e)) == hipErrorNotReady) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(50)) std::this_thread::yield();
  }
  if (q != hipSuccess) throw Error(GDSW_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
}

// Process-wide cache of device blocks, per device: the blocks of a destroyed
// context are handed to the next setup instead of being freed (hipMalloc and
// hipFree are slow and hipFree synchronizes the device).  A request takes the
// smallest cached block that fits with at most 25% slack; at most
// DEVICE_CACHE_LIMIT bytes stay cached, and none while less than a quarter of
// the device's memory is free (contexts alive beside each other, as in the
// serving loop, then get the memory instead of the cache).
constexpr size_t DEVICE_CACHE_LIMIT = size_t(64) << 30;
std::mutex g_dev_mu;
std::map<int, std::multimap<size_t, void*>> g_dev_free;
size_t g_dev_cached = 0;

void* device_take(size_t bytes, size_t& cap, int& dev) {
  GDSW_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> g(g_dev_mu);
    auto& m = g_dev_free[dev];
    auto it = m.lower_bound(bytes);
    if (it != m.end() && it->first <= bytes + bytes / 4) {
      cap = it->first;
      void* p = it->second;
      m.erase(it);
      g_dev_cached -= cap;
      return p;
    }
  }
  cap = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, cap);
  if (e == hipErrorOutOfMemory) {
    // blocks cached for reuse may be what fills the device: release this device's cache (no
    // context holds them) and try once more
    (void)hipGetLastError();
    std::vector<void*> drop;
    {
      std::lock_guard<std::mutex> g(g_dev_mu);
      auto& m = g_dev_free[dev];
      for (auto& kv : m) {
        drop.push_back(kv.second);
        g_dev_cached -= kv.first;
      }
      m.clear();
    }
    for (void* q : drop) (void)hipFree(q);
    e = hipMalloc(&p, cap);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(e == hipErrorOutOfMemory ? GDSW_ENOMEM : GDSW_EHIP,
                std::string("hipMalloc of ") + std::to_string(cap) + " bytes: " + hipGetErrorString(e));
  }
  return p;
}

// Whether device dev has at least a quarter of its memory free (only known for
// the current device; other devices count as having room).
bool device_has_room(int dev) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != dev) return true;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    return true;
  }
  return free_b >= total_b / 4;
}

// The caller guarantees that no queued work still uses p.
void device_give(void* p, size_t cap, int dev) {
  if (device_has_room(dev)) {
    std::lock_guard<std::mutex> g(g_dev_mu);
    if (g_dev_cached + cap <= DEVICE_CACHE_LIMIT) {
      g_dev_free[dev].emplace(cap, p);
      g_dev_cached += cap;
      return;
    }
  }
  (void)hipFree(p);
}

// Device memory owned by a context, taken from and returned to the cache above.
// Blocks go back on destroy, after the device has drained.
class Arena {
 public:
  ~Arena() { release(); }
  void* alloc(size_t bytes) {
    if (bytes == 0) bytes = 16;
    Block b;
    b.p = device_take(bytes, b.cap, b.dev);
    blocks_.push_back(b);
    bytes_ += bytes;
    return b.p;
  }
  template <typename T> T* alloc_n(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
  // Only for blocks no queued work uses any more.
  void free_one(void* p) {
    for (auto it = blocks_.begin(); it != blocks_.end(); ++it)
      if (it->p == p) {
        device_give(it->p, it->cap, it->dev);
        blocks_.erase(it);
        return;
      }
  }
  void release() {
    for (const Block& b : blocks_) device_give(b.p, b.cap, b.dev);
    blocks_.clear();
  }
  size_t bytes() const { return bytes_; }

 private:
  struct Block {
    void* p = nullptr;
    size_t cap = 0;
    int dev = 0;
  };
  std::vector<Block> blocks_;
  size_t bytes_ = 0;
};

// Page-locked host buffers shared by all contexts of the process; a context
// takes them while it uploads and gives them back at the end of its setup
// (held until the process exits).
std::mutex g_pin_mu;
std::multimap<size_t, void*> g_pin_free;

void* pinned_take(size_t bytes, size_t& cap) {
  {
    std::lock_guard<std::mutex> g(g_pin_mu);
    auto it = g_pin_free.lower_bound(bytes);
    if (it != g_pin_free.end()) {
      cap = it->first;
      void* p = it->second;
      g_pin_free.erase(it);
      return p;
    }
  }
  cap = std::max<size_t>(bytes, size_t(4) << 20);
  cap = (cap + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1);
  void* p = nullptr;
  GDSW_HIP(hipHostMalloc(&p, cap, hipHostMallocDefault));
  return p;
}

void pinned_give(void* p, size_t cap) {
  std::lock_guard<std::mutex> g(g_pin_mu);
  g_pin_free.emplace(cap, p);
}

// Copy n bytes with up to 16 host threads (large packs only).
void parallel_copy(char* dst, const char* src, size_t n) {
  constexpr size_t PIECE = size_t(1) << 20;
  if (n <= 2 * PIECE) {
    std::memcpy(dst, src, n);
    return;
  }
  const size_t pieces = (n + PIECE - 1) / PIECE;
  const int nt = (int)std::min<size_t>(pieces, (size_t)host_thread_count());
  std::atomic<size_t> next(0);
  host_parallel(nt, [&](int) {
    for (;;) {
      const size_t k = next.fetch_add(1);
      if (k >= pieces) break;
      const size_t o = k * PIECE;
      std::memcpy(dst + o, src + o, std::min(PIECE, n - o));
    }
  });
}

struct Level {
  int index = 0;                 // 1-based level number
  int nparts = 0;
  int64_t n = 0;                 // rows of this level's operator
  CsrDev K;
  LevelMaps maps;
  // local blocks
  int max_n = 0;
  int64_t sum_n = 0, sum_n2 = 0;  // sum_n2: elements of the stored blocks (n_i x lead_dim(n_i, pad))
  int pad = 1;                     // block columns padded to 128 bytes
  std::vector<int> dims;
  std::vector<int> order_h;
  std::vector<int64_t> blk_off_h;
  int64_t* dom_ptr = nullptr;
  int* dom = nullptr;
  int64_t* blk_off = nullptr;
  int* dim = nullptr;
  void* blocks = nullptr;        // double or float
  int* piv = nullptr;
  int* perm = nullptr;
  int* gidx = nullptr;
  int* info = nullptr;
  int* order = nullptr;          // parts by decreasing block size (apply visiting order)
  int64_t* tmask_off = nullptr;  // per part: offset of its nonzero-tile masks (see tile_masks)
  unsigned long long* tmask = nullptr;
  unsigned long long* tkept = nullptr;  // factor elements the masked substitution reads
  int ls_waves = 8;              // wavefronts per matrix of the local solves (2, 4 or 8); autotuned
                                 // with tune = 1
  int64_t* sc_ptr = nullptr;
  int* sc_pos = nullptr;
  double* w = nullptr;           // local solutions, sum_n
  // coarse space (absent on the last Schwarz level when the coarsest correction is dropped)
  bool has_coarse = false;
  int n_coarse = 0;
  int64_t* int_ptr = nullptr;
  int* inter = nullptr;
  int* dof_gcol = nullptr;
  int* dof_ipart = nullptr;
  int* dof_irow = nullptr;
  int64_t* pc_ptr = nullptr;
  int* pcols = nullptr;
  int64_t* cp_ptr = nullptr;
  int* cp_part = nullptr;
  int* cp_lc = nullptr;
  int64_t* col_ptr = nullptr;
  int* col_dofs = nullptr;
  int64_t* phi_off = nullptr;
  void* phi = nullptr;           // double or float, |I_i| x m_i column-major per part
  int* iinfo = nullptr;
  int* gdofs = nullptr;          // interface dofs (rows of Phi_Gamma)
  int64_t n_gdofs = 0;
  int max_m = 0;                 // largest number of coarse columns of a part
  int* bad = nullptr;            // set by the basis/Galerkin kernels on non-element-local couplings
  int max_ni = 0;
  double* rc = nullptr;          // restricted residual (n_coarse)
  double* yc = nullptr;          // coarse correction (n_coarse)
  double interior_flops = 0.0;
  int64_t phi_elems = 0;         // sum_i |I_i| m_i (values of Phi_I)
  // several right-hand sides (gdsw_apply_multi): local solutions [s][sum_n], coarse vectors [s][n_coarse]
  int multi_cap = 0;
  double* wm = nullptr;
  double* rcm = nullptr;
  double* ycm = nullptr;
  hipEvent_t lu_ev[2] = {nullptr, nullptr};   // around the batched LU of this level (timing)
  int lu_variant = 0;            // LU variant: bit 0 = single steps, bit 1 = full-width panels,
                                 // bit 2 = size-classed register panels
};

}  // namespace

}  // namespace gdsw

struct gdsw_ctx {
  gdsw::Arena arena;
  gdsw_options opt;
  int mixed = 0;
  std::vector<gdsw::Level> levels;     // Schwarz levels
  bool has_coarsest = false;
  int nc = 0;                          // coarsest order
  double* ainv = nullptr;              // coarsest inverse (column-major)
  double* gemv_partial = nullptr;
  int64_t nnz_coarsest = 0;
  gdsw_stats stats;
  // FGMRES workspace
  int ws_m = -1;
  hipEvent_t ev_fetch = nullptr;       // Hessenberg column copied to the host
  double *V = nullptr, *Z = nullptr, *wv = nullptr, *dpart = nullptr, *hdev = nullptr, *ydev = nullptr;
  double* hhost = nullptr;
  // host-side Givens/Hessenberg arrays of the solve, sized at setup for the restart length
  std::vector<double> kH, kcs, ksn, kg, ky;
  bool no_alloc_call = false;          // inside gdsw_solve_noalloc: no event creation in applies
  // gdsw_solve_multi: workspaces of up to multi_cap systems, page-locked Hessenberg columns
  int multi_cap = 0, multi_m = -1;
  double *mV = nullptr, *mZ = nullptr, *mW = nullptr, *mH = nullptr, *mY = nullptr, *mP = nullptr;
  double* mhost = nullptr;
  // event pairs around level-1 local-solve launches (profile = 1)
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_level;           // level (0-based) of each event pair
  size_t ev_used = 0;
  // the coarse chain of the apply runs on `side`, forked from and joined to the caller's stream;
  // during setup `side` factors level 1 and `side2` the deeper levels
  hipStream_t side = nullptr, side2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_fork2 = nullptr, ev_join2 = nullptr;   // level 2's coarse chain on side2
  // host-to-device uploads run on `up`, which never holds compute work
  hipStream_t up = nullptr;
  hipEvent_t ev_up = nullptr;
  // graph mode: the solve runs on `own`; apply graphs per Krylov column
  hipStream_t own = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<hipGraphExec_t> apply_exec;
  bool capturing = false;
  // device scratch needed only during setup (returned to the block cache at its end)
  std::vector<void*> setup_scratch;
  // page-locked staging buffers held while uploads may be in flight
  std::vector<std::pair<void*, size_t>> pinned;
  // an event recorded on every caller stream after each call: gdsw_destroy waits for these (and
  // the context's own streams) instead of the whole device
  std::map<hipStream_t, hipEvent_t> stream_marks;
  void release_pinned() {
    for (auto& pc : pinned) gdsw::pinned_give(pc.first, pc.second);
    pinned.clear();
  }
  ~gdsw_ctx() {
    if (own) (void)hipStreamSynchronize(own);
    for (gdsw::Level& L : levels)
      for (hipEvent_t e : L.lu_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipGraphExec_t g : apply_exec)
      if (g) (void)hipGraphExecDestroy(g);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (own) (void)hipStreamDestroy(own);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_fork2) (void)hipEventDestroy(ev_fork2);
    if (ev_join2) (void)hipEventDestroy(ev_join2);
    if (side) {
      (void)hipStreamSynchronize(side);
      (void)hipStreamDestroy(side);
    }
    if (side2) {
      (void)hipStreamSynchronize(side2);
      (void)hipStreamDestroy(side2);
    }
    if (up) {
      (void)hipStreamSynchronize(up);
      (void)hipStreamDestroy(up);
    }
    release_pinned();
    for (auto& kv : stream_marks) {
      (void)hipEventSynchronize(kv.second);
      (void)hipEventDestroy(kv.second);
    }
    if (hhost) (void)hipHostFree(hhost);
    if (mhost) (void)hipHostFree(mhost);
    if (ev_up) (void)hipEventDestroy(ev_up);
    if (ev_fetch) (void)hipEventDestroy(ev_fetch);
  }
};

namespace gdsw {
namespace {

// Make stream s wait for every upload issued so far.
void wait_uploads(gdsw_ctx* C, hipStream_t s) {
  GDSW_HIP(hipEventRecord(C->ev_up, C->up));
  GDSW_HIP(hipStreamWaitEvent(s, C->ev_up, 0));
}

// Uploads of one setup phase: the host arrays are packed into one page-locked
// buffer and moved with a single asynchronous copy on the upload stream into
// one device allocation; each destination pointer is set to its slice.
class UploadBatch {
 public:
  template <typename T, typename A>
  void add(T** dst, const std::vector<T, A>& v) {
    entries_.push_back({reinterpret_cast<void**>(dst), v.data(), v.size() * sizeof(T), total_});
    total_ += (v.size() * sizeof(T) + 255) & ~size_t(255);
  }
  // Pack, copy and point the destinations at the device slices; stream s then
  // waits for the copy.
  void flush(gdsw_ctx* C, hipStream_t s) {
    if (entries_.empty()) return;
    const size_t total = std::max<size_t>(total_, 256);
    char* d = static_cast<char*>(C->arena.alloc(total));
    size_t cap = 0;
    char* h = static_cast<char*>(pinned_take(total, cap));
    C->pinned.push_back({h, cap});
    for (const Entry& e : entries_) {
      if (e.bytes) parallel_copy(h + e.off, static_cast<const char*>(e.src), e.bytes);
      *e.dst = d + e.off;
    }
    GDSW_HIP(hipMemcpyAsync(d, h, total_, hipMemcpyHostToDevice, C->up));
    wait_uploads(C, s);
    entries_.clear();
    total_ = 0;
  }

 private:
  struct Entry {
    void** dst;
    const void* src;
    size_t bytes, off;
  };
  std::vector<Entry> entries_;
  size_t total_ = 0;
};

int64_t checked_i32(int64_t v, const char* what) {
  if (v > INT32_MAX) throw Error(GDSW_EINVAL, std::string(what) + " exceeds the int32 index range");
  return v;
}

// Tuning results shared by all contexts of the process, keyed by what decides
// the choice: the value type, the level and the batch shape (count, total and
// largest order of the local blocks).  With GDSW_TUNE_CACHE=<file> the table is
// read from that file on first use and every new entry is appended to it, so
// later processes skip the timing runs.
struct TuneCache {
  std::mutex mu;
  bool loaded = false;
  std::map<std::string, int> waves;
};
TuneCache& tune_cache() {
  static TuneCache c;
  return c;
}
std::string tune_key(const char* tag, int value_bytes, int level, int nparts, int64_t sum_n, int max_n) {
  return std::string(tag) + " " + std::to_string(value_bytes) + " " + std::to_string(level) + " " +
         std::to_string(nparts) + " " + std::to_string(sum_n) + " " + std::to_string(max_n);
}
bool tune_lookup(const std::string& key, int* w) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  if (!c.loaded) {
    c.loaded = true;
    if (const char* path = std::getenv("GDSW_TUNE_CACHE")) {
      if (FILE* f = std::fopen(path, "r")) {
        char tag[8];
        int vb, lv, np, mx, wv;
        long long sn;
        while (std::fscanf(f, "%7s %d %d %d %lld %d %d", tag, &vb, &lv, &np, &sn, &mx, &wv) == 7) {
          const std::string t(tag);
          if ((t == "ls" && (wv == 2 || wv == 4 || wv == 8)) || (t == "lu" && wv >= 0 && wv <= 7))
            c.waves[tune_key(tag, vb, lv, np, sn, mx)] = wv;
        }
        std::fclose(f);
      }
    }
  }
  auto it = c.waves.find(key);
  if (it == c.waves.end()) return false;
  *w = it->second;
  return true;
}
void tune_store(const std::string& key, int w) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.waves[key] = w;
  if (const char* path = std::getenv("GDSW_TUNE_CACHE")) {
    if (FILE* f = std::fopen(path, "a")) {
      std::fprintf(f, "%s %d\n", key.c_str(), w);
      std::fclose(f);
    }
  }
}

template <typename T>
void factor_level(gdsw_ctx* C, Level& L, hipStream_t s) {
  const double th = now_ms();
  Arena& A = C->arena;
  const LevelMaps& m = L.maps;
  const int N = L.nparts;
  L.dims.resize(N);
  L.blk_off_h.resize(N);
  L.max_n = 0;
  L.sum_n = 0;
  L.sum_n2 = 0;
  L.pad = (int)(128 / sizeof(T));
  for (int i = 0; i < N; ++i) {
    const int ni = (int)(m.dom_ptr[i + 1] - m.dom_ptr[i]);
    L.dims[i] = ni;
    L.blk_off_h[i] = L.sum_n2;
    L.sum_n2 += (int64_t)ni * lead_dim(ni, L.pad);
    L.sum_n += ni;
    L.max_n = std::max(L.max_n, ni);
  }
  L.order_h.resize(N);
  for (int i = 0; i < N; ++i) L.order_h[i] = i;
  std::stable_sort(L.order_h.begin(), L.order_h.end(), [&](int a, int b) { return L.dims[a] > L.dims[b]; });
  // ordered combination lists: every position holding g (additive) or the owner's only (restricted)
  std::vector<int64_t> sc_ptr;
  std::vector<int> sc_pos;
  const std::string err = scatter_lists(m, L.n, C->opt.combine == GDSW_COMBINE_ADDITIVE, sc_ptr, sc_pos);
  if (!err.empty()) throw Error(GDSW_EINVAL, err);
  // tile masks: ceil(nt / 64) 64-bit words per 64-column panel (nt panels per block)
  std::vector<int64_t> tmask_off(N);
  int64_t tmask_words = 0;
  for (int i = 0; i < N; ++i) {
    const int64_t nt = (L.dims[i] + 63) / 64;
    tmask_off[i] = tmask_words;
    tmask_words += nt * ((nt + 63) / 64);
  }
  LuTiles tiles;
  tiles.build(L.dims.data(), N);
  int64_t *d_tiles_outer, *d_tiles_inner;
  UploadBatch B;
  B.add(&d_tiles_outer, tiles.outer);
  B.add(&d_tiles_inner, tiles.inner);
  B.add(&L.dom_ptr, m.dom_ptr);
  B.add(&L.dom, m.dom);
  B.add(&L.blk_off, L.blk_off_h);
  B.add(&L.order, L.order_h);
  B.add(&L.dim, L.dims);
  B.add(&L.tmask_off, tmask_off);
  if (!sc_ptr.empty()) B.add(&L.sc_ptr, sc_ptr);
  B.add(&L.sc_pos, sc_pos);
  B.flush(C, s);
  C->stats.ms_extract += now_ms() - th;     // host-side preparation of the level (lists and uploads)
  T* blocks = A.alloc_n<T>((size_t)L.sum_n2);
  L.blocks = blocks;
  GDSW_HIP(hipMemsetAsync(blocks, 0, (size_t)L.sum_n2 * sizeof(T), s));
  extract_blocks<T>(L.K, N, L.max_n, L.order, L.dom_ptr, L.dom, L.blk_off, blocks, L.pad, s);
  L.piv = A.alloc_n<int>((size_t)L.sum_n);
  L.info = A.alloc_n<int>(N);
  GDSW_HIP(hipMemsetAsync(L.info, 0, N * sizeof(int), s));
  LuBatch b;
  b.count = N;
  b.max_n = L.max_n;
  b.off = L.blk_off;
  b.dim = L.dim;
  b.piv = L.piv;
  b.poff = L.dom_ptr;
  b.info = L.info;
  b.pad = L.pad;
  b.tiles_outer = d_tiles_outer;
  b.tiles_inner = d_tiles_inner;
  b.total_outer = tiles.total_outer.data();
  b.total_inner = tiles.total_inner.data();
  b.wide = true;
  b.ut = A.alloc_n<T>((size_t)128 * L.sum_n);
  C->setup_scratch.push_back(b.ut);
  b.step_masks = A.alloc_n<unsigned long long>((size_t)2 * N);
  C->setup_scratch.push_back(b.step_masks);
  std::vector<int> sorted_dims(N);
  for (int q = 0; q < N; ++q) sorted_dims[q] = L.dims[L.order_h[q]];
  b.order = L.order;
  b.order_dims = sorted_dims.data();
  auto set_variant = [&](int v) {
    b.wide = (v & 1) == 0;
    b.full_panels = (v >> 1) & 1;
    b.panel_classes = (v >> 2) & 1;
  };
  if (C->opt.tune & 2) {
    // LU autotuner: paired 64-column steps with rank-128 trailing updates or single steps with
    // rank-64 updates, half-width or full-width register panels for FP64 panels of 769..2048
    // rows; each variant factors the level's blocks once (re-extracted before each trial), the
    // fastest is kept for this batch shape (process-wide, and in GDSW_TUNE_CACHE if set).
    const std::string key = tune_key("lu", (int)sizeof(T), L.index, N, L.sum_n, L.max_n);
    int variant = 0;
    if (!tune_lookup(key, &variant)) {
      hipEvent_t t0, t1;
      GDSW_HIP(hipEventCreate(&t0));
      GDSW_HIP(hipEventCreate(&t1));
      float best = 1e30f;
      for (int v = 0; v < 8; ++v) {
        if (sizeof(T) == 4 && (v & 2)) continue;     // full-width panels: an FP64 choice only
        set_variant(v);
        GDSW_HIP(hipMemsetAsync(blocks, 0, (size_t)L.sum_n2 * sizeof(T), s));
        extract_blocks<T>(L.K, N, L.max_n, L.order, L.dom_ptr, L.dom, L.blk_off, blocks, L.pad, s);
        GDSW_HIP(hipEventRecord(t0, s));
        lu_batched<T>(b, blocks, s);
        GDSW_HIP(hipEventRecord(t1, s));
        GDSW_HIP(hipEventSynchronize(t1));
        float ms = 0;
        GDSW_HIP(hipEventElapsedTime(&ms, t0, t1));
        if (ms < best) {
          best = ms;
          variant = v;
        }
      }
      (void)hipEventDestroy(t0);
      (void)hipEventDestroy(t1);
      tune_store(key, variant);
      GDSW_HIP(hipMemsetAsync(blocks, 0, (size_t)L.sum_n2 * sizeof(T), s));
      extract_blocks<T>(L.K, N, L.max_n, L.order, L.dom_ptr, L.dom, L.blk_off, blocks, L.pad, s);
      GDSW_HIP(hipMemsetAsync(L.info, 0, N * sizeof(int), s));
    }
    set_variant(variant);
    L.lu_variant = variant;
  } else {
    set_variant(C->opt.lu_variant);
    L.lu_variant = C->opt.lu_variant;
  }
  GDSW_HIP(hipEventCreate(&L.lu_ev[0]));
  GDSW_HIP(hipEventCreate(&L.lu_ev[1]));
  GDSW_HIP(hipEventRecord(L.lu_ev[0], s));
  lu_batched<T>(b, blocks, s);
  GDSW_HIP(hipEventRecord(L.lu_ev[1], s));
  L.tmask = A.alloc_n<unsigned long long>((size_t)std::max<int64_t>(1, tmask_words));
  L.tkept = A.alloc_n<unsigned long long>(1);
  GDSW_HIP(hipMemsetAsync(L.tmask, 0, (size_t)std::max<int64_t>(1, tmask_words) * sizeof(unsigned long long), s));
  GDSW_HIP(hipMemsetAsync(L.tkept, 0, sizeof(unsigned long long), s));
  tile_masks<T>(N, L.dom_ptr, L.blk_off, blocks, L.pad, L.tmask_off, L.tmask, L.tkept, s);
  L.perm = A.alloc_n<int>((size_t)L.sum_n);
  lu_build_perm(b, L.perm, s);
  L.gidx = A.alloc_n<int>((size_t)L.sum_n);
  make_gather_index(N, L.sum_n, L.dom_ptr, L.dom, L.perm, L.gidx, s);
  L.w = A.alloc_n<double>((size_t)L.sum_n);
}

// GDSW basis of the level and the Galerkin operator of the next one.
template <typename T>
CsrDev coarse_level(gdsw_ctx* C, Level& L, hipStream_t s, std::vector<int64_t>& a0_rowptr_h,
                    std::vector<int>& a0_col_h) {
  const double th = now_ms();
  Arena& A = C->arena;
  const LevelMaps& m = L.maps;
  const int N = L.nparts;
  L.has_coarse = true;
  L.n_coarse = m.n_coarse;
  int64_t *z_ptr, *d_aii_off, *d_v_off, *d_c_off;
  int *z_dof, *z_lc, *d_ni, *d_mi;
  UploadBatch B;
  B.add(&L.int_ptr, m.int_ptr);
  B.add(&L.inter, m.inter);
  B.add(&L.dof_gcol, m.dof_gcol);
  B.add(&L.dof_ipart, m.dof_ipart);
  B.add(&L.dof_irow, m.dof_irow);
  B.add(&L.pc_ptr, m.pc_ptr);
  B.add(&L.pcols, m.pcols);
  B.add(&L.cp_ptr, m.cp_ptr);
  B.add(&L.cp_part, m.cp_part);
  B.add(&L.cp_lc, m.cp_lc);
  B.add(&L.col_ptr, m.col_ptr);
  B.add(&L.col_dofs, m.col_dofs);
  B.add(&z_ptr, m.z_ptr);
  B.add(&z_dof, m.z_dof);
  B.add(&z_lc, m.z_lc);
  std::vector<int64_t> aii_off(N), phi_off(N + 1), v_off(N), c_off(N);
  std::vector<int> ni(N), mi(N);
  int64_t aii_tot = 0, phi_tot = 0, v_tot = 0, c_tot = 0;
  int max_ni = 0, max_m = 0;
  double iflops = 0.0;
  for (int i = 0; i < N; ++i) {
    const int nI = (int)(m.int_ptr[i + 1] - m.int_ptr[i]);
    const int mm = (int)(m.pc_ptr[i + 1] - m.pc_ptr[i]);
    const int nZ = (int)(m.z_ptr[i + 1] - m.z_ptr[i]);
    ni[i] = nI;
    mi[i] = mm;
    aii_off[i] = aii_tot;
    aii_tot += (int64_t)nI * nI;
    phi_off[i] = phi_tot;
    phi_tot += (int64_t)nI * mm;
    v_off[i] = v_tot;
    v_tot += (int64_t)nZ * mm;
    c_off[i] = c_tot;
    c_tot += (int64_t)mm * mm;
    max_ni = std::max(max_ni, nI);
    max_m = std::max(max_m, mm);
    iflops += (2.0 / 3.0) * nI * (double)nI * nI + 2.0 * nI * (double)nI * mm;
  }
  phi_off[N] = phi_tot;
  L.max_ni = max_ni;
  L.max_m = max_m;
  L.interior_flops = iflops;
  L.phi_elems = phi_tot;
  std::vector<int> gd;
  for (int64_t g = 0; g < L.n; ++g)
    if (m.dof_gcol[g] >= 0) gd.push_back((int)g);
  L.n_gdofs = (int64_t)gd.size();
  B.add(&L.gdofs, gd);
  B.add(&d_aii_off, aii_off);
  B.add(&L.phi_off, phi_off);
  B.add(&d_v_off, v_off);
  B.add(&d_c_off, c_off);
  B.add(&d_ni, ni);
  B.add(&d_mi, mi);
  LuTiles itiles;
  itiles.build(ni.data(), N);
  int64_t *d_itiles_outer, *d_itiles_inner;
  B.add(&d_itiles_outer, itiles.outer);
  B.add(&d_itiles_inner, itiles.inner);
  B.flush(C, s);
  C->stats.ms_extract += now_ms() - th;
  T* aii = A.alloc_n<T>((size_t)aii_tot);
  GDSW_HIP(hipMemsetAsync(aii, 0, (size_t)aii_tot * sizeof(T), s));
  double* rhs = A.alloc_n<double>((size_t)phi_tot);
  GDSW_HIP(hipMemsetAsync(rhs, 0, (size_t)phi_tot * sizeof(double), s));
  int* bad = A.alloc_n<int>(1);
  GDSW_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  L.bad = bad;
  extract_interior<T>(L.K, N, (int64_t)m.inter.size(), L.int_ptr, L.inter, L.dof_ipart, L.dof_irow, L.dof_gcol,
                      L.pc_ptr, L.pcols, d_aii_off, aii, L.phi_off, rhs, bad, s);
  int* ipiv = A.alloc_n<int>(m.inter.size());
  L.iinfo = A.alloc_n<int>(N);
  GDSW_HIP(hipMemsetAsync(L.iinfo, 0, N * sizeof(int), s));
  LuBatch b;
  b.count = N;
  b.max_n = max_ni;
  b.off = d_aii_off;
  b.dim = d_ni;
  b.piv = ipiv;
  b.poff = L.int_ptr;
  b.info = L.iinfo;
  b.tiles_outer = d_itiles_outer;
  b.tiles_inner = d_itiles_inner;
  b.total_outer = itiles.total_outer.data();
  b.total_inner = itiles.total_inner.data();
  b.wide = true;
  b.ut = A.alloc_n<T>((size_t)128 * m.inter.size());
  C->setup_scratch.push_back(b.ut);
  b.step_masks = A.alloc_n<unsigned long long>((size_t)2 * N);
  C->setup_scratch.push_back(b.step_masks);
  lu_batched<T>(b, aii, s);
  T* phi;
  if (sizeof(T) == sizeof(double)) {
    phi = reinterpret_cast<T*>(rhs);
  } else {
    phi = A.alloc_n<T>((size_t)phi_tot);
    convert<double, T>(rhs, phi, phi_tot, s);
  }
  lu_solve_batched<T>(b, aii, phi, L.phi_off, d_mi, max_m, s);
  L.phi = phi;
  // Galerkin product
  double* W = A.alloc_n<double>((size_t)phi_tot);
  double* V = A.alloc_n<double>((size_t)v_tot);
  double* Cm = A.alloc_n<double>((size_t)c_tot);
  T* phit = A.alloc_n<T>((size_t)std::max<int64_t>(phi_tot, 1));
  C->setup_scratch.push_back(phit);
  galerkin_wv<T>(L.K, N, (int64_t)m.inter.size(), (int64_t)m.z_dof.size(), L.int_ptr, L.inter, L.dof_ipart,
                 L.dof_irow, L.dof_gcol, L.pc_ptr, L.pcols, L.phi_off, phi, phit, z_ptr, z_dof, d_v_off, W, V, bad,
                 s);
  galerkin_local<T>(N, (int64_t)m.pcols.size(), L.int_ptr, L.pc_ptr, L.phi_off, phi, W, z_ptr, z_lc, d_v_off, V,
                    d_c_off, Cm, s);
  // sparsity of the coarse operator, built on the host while the kernels above run
  const double tp = now_ms();
  coarse_pattern(m, a0_rowptr_h, a0_col_h);
  int max_row = 0;
  for (int c = 0; c < m.n_coarse; ++c) max_row = std::max(max_row, (int)(a0_rowptr_h[c + 1] - a0_rowptr_h[c]));
  int64_t* rp;
  int* cl;
  B.add(&rp, a0_rowptr_h);
  B.add(&cl, a0_col_h);
  B.flush(C, s);
  C->stats.ms_extract += now_ms() - tp;

  CsrDev K0;
  K0.n = m.n_coarse;
  K0.nnz = (int64_t)a0_col_h.size();

  double* val = A.alloc_n<double>((size_t)K0.nnz);
  galerkin_assemble(L.K, L.col_ptr, L.col_dofs, L.dof_gcol, L.cp_ptr, L.cp_part, L.cp_lc, L.pc_ptr, L.pcols, d_c_off,
                    Cm, rp, cl, val, m.n_coarse, max_row, bad, s);
  K0.rowptr = rp;
  K0.col = cl;
  K0.val = val;
  L.rc = A.alloc_n<double>(m.n_coarse);
  L.yc = A.alloc_n<double>(m.n_coarse);
  return K0;
}

void coarsest_inverse(gdsw_ctx* C, const CsrDev& K, hipStream_t s, double** dense_out, int** info_out) {
  Arena& A = C->arena;
  const int n = (int)K.n;
  C->nc = n;
  double* D = A.alloc_n<double>((size_t)n * n);
  GDSW_HIP(hipMemsetAsync(D, 0, (size_t)n * n * sizeof(double), s));
  csr_to_dense(K, D, s);
  // a batch of one: offset 0, order n (set on the device, nothing to upload)
  int64_t* d_off = A.alloc_n<int64_t>(1);
  int* d_dim = A.alloc_n<int>(1);
  GDSW_HIP(hipMemsetAsync(d_off, 0, sizeof(int64_t), s));
  GDSW_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(d_dim), n, 1, s));
  int* piv = A.alloc_n<int>(n);
  int* info = A.alloc_n<int>(1);
  GDSW_HIP(hipMemsetAsync(info, 0, sizeof(int), s));
  LuBatch b;
  b.count = 1;
  b.max_n = n;
  b.off = d_off;
  b.dim = d_dim;
  b.piv = piv;
  b.poff = d_off;
  b.info = info;
  b.wide = true;
  b.ut = A.alloc_n<double>((size_t)128 * n);
  C->setup_scratch.push_back(b.ut);
  b.tall_scratch = A.alloc(lu_tall_scratch_bytes(n, sizeof(double)));
  C->setup_scratch.push_back(b.tall_scratch);
  lu_batched<double>(b, D, s);
  double* X = A.alloc_n<double>((size_t)n * n);
  // the inverse is kept by rows, so the per-apply GEMV reads rows contiguously
  int* perm = A.alloc_n<int>(n);
  lu_build_perm(b, perm, s);
  if (lu_inverse_transposed(D, perm, X, n, s)) {
    C->ainv = X;                 // D (the factors) becomes scratch
  } else {
    int* iscr = A.alloc_n<int>((size_t)2 * n + 64);
    C->setup_scratch.push_back(iscr);
    lu_inverse_blocked(b, D, perm, X, iscr, n, s);
    transpose_square(n, X, D, s);
    C->ainv = D;
    D = X;
  }
  *dense_out = D;
  *info_out = info;
}

void check_info(const int* dinfo, int N, const std::string& what, int level, hipStream_t) {
  std::vector<int> h(N);
  GDSW_HIP(hipMemcpy(h.data(), dinfo, N * sizeof(int), hipMemcpyDeviceToHost));
  for (int i = 0; i < N; ++i)
    if (h[i] != 0)
      throw Error(GDSW_ESINGULAR, what + " of level " + std::to_string(level) + ", part " + std::to_string(i) +
                                      " has a zero pivot at column " + std::to_string(h[i] - 1));
}

struct Plan {
  std::vector<LevelMesh> meshes;
  std::vector<LevelMaps> maps;
  int schwarz = 0;        // levels with local solves
  bool coarsest = false;  // a direct coarsest level follows
};

void validate_problem(const gdsw_problem* p) {
  if (!p) throw Error(GDSW_EINVAL, "problem is NULL");
  if (p->levels < 2 || p->levels > 8) throw Error(GDSW_EINVAL, "levels must be in [2, 8]");
  if (!p->n_parts || !p->node_dof || !p->elem_node || !p->elem_pdof || !p->elem_part)
    throw Error(GDSW_EINVAL, "a required host array is NULL");
  if (p->levels > 2 && !p->part_parent) throw Error(GDSW_EINVAL, "part_parent is NULL");
}

Plan plan_levels(const gdsw_problem* p, const gdsw_options& o) {
  validate_problem(p);
  Plan P;
  P.meshes.emplace_back();
  std::string err = build_level1_mesh(p->n, p->n_nodes, p->node_dof, p->n_elem, p->elem_node, p->elem_pdof,
                                      p->elem_part, p->n_parts[0], P.meshes[0]);
  if (!err.empty()) throw Error(GDSW_EINVAL, err);
  const int L = p->levels;
  for (int l = 1; l < L; ++l) {
    P.maps.emplace_back();
    build_maps(P.meshes[l - 1], o.overlap, P.maps.back(), o.pressure_gamma == 0);
    P.schwarz = l;
    const bool last = (l == L - 1);
    if (last) {
      P.coarsest = !o.no_coarse;
      break;
    }
    if (P.maps.back().n_coarse == 0) throw Error(GDSW_EINVAL, "coarse space of level " + std::to_string(l) + " is empty");
    const int nxt = p->n_parts[l];
    if (nxt <= 0) throw Error(GDSW_EINVAL, "n_parts must be positive");
    P.meshes.emplace_back();
    err = build_next_mesh(P.meshes[l - 1], P.maps.back(), p->part_parent[l - 1], nxt, P.meshes[l]);
    if (!err.empty()) throw Error(GDSW_EINVAL, err);
    if (nxt == 1) {          // a single part: this coarse problem becomes the coarsest
      P.coarsest = true;
      break;
    }
  }
  if (P.coarsest && P.maps.back().n_coarse == 0) throw Error(GDSW_EINVAL, "coarsest space is empty");
  return P;
}

// Host maps of level l+1 are built while the GPU works on level l: every
// launch is asynchronous and the pivot / consistency flags are checked once,
// after the last level.
template <typename T>
void setup_impl(gdsw_ctx* C, const gdsw_problem* p, hipStream_t s) {
  const double t0 = now_ms();
  gdsw_stats& st = C->stats;
  std::memset(&st, 0, sizeof(st));
  validate_problem(p);
  double host_ms = 0;
  auto host = [&](auto&& fn) {
    const double a = now_ms();
    fn();
    host_ms += now_ms() - a;
  };
  std::vector<LevelMesh> meshes(1);
  host([&] {
    std::string err = build_level1_mesh(p->n, p->n_nodes, p->node_dof, p->n_elem, p->elem_node, p->elem_pdof,
                                        p->elem_part, p->n_parts[0], meshes[0]);
    if (!err.empty()) throw Error(GDSW_EINVAL, err);
  });
  // level-1 operator: a private copy of the caller's CSR
  CsrDev K;
  K.n = p->n;
  unsigned long long* saved3 = nullptr;
  int64_t nnz = 0;
  GDSW_HIP(hipMemcpyAsync(&nnz, p->rowptr + p->n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  GDSW_HIP(hipStreamSynchronize(s));
  if (nnz <= 0) throw Error(GDSW_EINVAL, "K has no nonzero");
  K.nnz = nnz;
  {
    int64_t* rp = C->arena.alloc_n<int64_t>(p->n + 1);
    int* cl = C->arena.alloc_n<int>((size_t)nnz);
    double* vl = C->arena.alloc_n<double>((size_t)nnz);
    GDSW_HIP(hipMemcpyAsync(rp, p->rowptr, (p->n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    GDSW_HIP(hipMemcpyAsync(cl, p->col, nnz * sizeof(int), hipMemcpyDeviceToDevice, s));
    GDSW_HIP(hipMemcpyAsync(vl, p->val, nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    K.rowptr = rp;
    K.col = cl;
    K.val = vl;
    // groups of three rows with one column list (a node's velocity components) for the SpMV
    unsigned char* same3 = C->arena.alloc_n<unsigned char>((size_t)(p->n + 2) / 3);
    saved3 = C->arena.alloc_n<unsigned long long>(1);
    C->setup_scratch.push_back(saved3);
    GDSW_HIP(hipMemsetAsync(saved3, 0, sizeof(unsigned long long), s));
    spmv_groups3(K, same3, saved3, s);
    K.same3 = same3;
  }
  const int Lp = p->levels;
  C->levels.reserve(Lp);
  std::vector<hipEvent_t> evs;
  auto mark = [&](hipStream_t st_) {
    hipEvent_t e;
    GDSW_HIP(hipEventCreate(&e));
    GDSW_HIP(hipEventRecord(e, st_));
    evs.push_back(e);
    return (int)evs.size() - 1;
  };
  const int e_setup = mark(s);
  // The local factorizations run on side streams (level 1 on one, deeper
  // levels on another), concurrently with the basis / Galerkin / coarser-level
  // chain on the caller's stream; level l's factorization only waits for its
  // operator K_l.
  std::vector<std::pair<int, int>> ev_factor, ev_basis;
  bool coarsest = false;
  int k_ready = mark(s);                      // K_1 copied
  for (int l = 0; l < Lp - 1; ++l) {
    C->levels.emplace_back();
    Level& L = C->levels.back();
    L.index = l + 1;
    L.ls_waves = C->opt.ls_waves ? C->opt.ls_waves : 8;
    L.nparts = meshes[l].n_parts;
    L.n = K.n;
    L.K = K;
    // the overlapping sets first: the local factorizations start while the
    // host builds the rest of the level's maps
    host([&] { build_domains(meshes[l], C->opt.overlap, L.maps); });
    hipStream_t fs = (l == 0) ? C->side : C->side2;
    GDSW_HIP(hipStreamWaitEvent(fs, evs[k_ready], 0));
    const int e0 = mark(fs);
    factor_level<T>(C, L, fs);
    ev_factor.push_back({e0, mark(fs)});
    host([&] { build_maps(meshes[l], C->opt.overlap, L.maps, C->opt.pressure_gamma == 0); });
    st.n[l] = L.n;
    st.parts[l] = L.nparts;
    st.sum_ni[l] = L.sum_n;
    st.max_ni[l] = L.max_n;
    st.factor_bytes[l] = L.sum_n2 * (int64_t)sizeof(T);
    st.nnz[l] = K.nnz;
    double f = 0;
    for (int d : L.dims) f += (2.0 / 3.0) * d * (double)d * d;
    st.factor_flops[l] = f;
    const bool last = (l == Lp - 2);
    if (last && C->opt.no_coarse) break;
    if (L.maps.n_coarse == 0) throw Error(GDSW_EINVAL, "coarse space of level " + std::to_string(l + 1) + " is empty");
    int nxt = 0;
    if (!last) {
      nxt = p->n_parts[l + 1];
      if (nxt <= 0) throw Error(GDSW_EINVAL, "n_parts must be positive");
    }
    std::vector<int64_t> rp;
    std::vector<int> cl;
    const int b0 = mark(s);
    K = coarse_level<T>(C, L, s, rp, cl);
    k_ready = mark(s);
    ev_basis.push_back({b0, k_ready});
    st.interior_flops[l] = L.interior_flops;
    if (last || nxt == 1) {          // a single coarse part: that coarse problem is the coarsest
      coarsest = true;
      break;
    }
    meshes.emplace_back();
    host([&] {
      std::string err = build_next_mesh(meshes[l], L.maps, p->part_parent[l], nxt, meshes[l + 1]);
      if (!err.empty()) throw Error(GDSW_EINVAL, err);
    });
  }
  const int schwarz = (int)C->levels.size();
  st.levels = schwarz + (coarsest ? 1 : 0);
  int ec0 = -1, ec1 = -1;
  double* dense = nullptr;
  int* cinfo = nullptr;
  if (coarsest) {
    C->has_coarsest = true;
    C->nnz_coarsest = K.nnz;
    ec0 = mark(s);
    coarsest_inverse(C, K, s, &dense, &cinfo);
    ec1 = mark(s);
    st.n[schwarz] = K.n;
    st.nnz[schwarz] = K.nnz;
    st.factor_flops[schwarz] = (2.0 / 3.0) * K.n * (double)K.n * K.n + 2.0 * K.n * (double)K.n * K.n;
  }
  GDSW_HIP(hipStreamSynchronize(C->side));
  GDSW_HIP(hipStreamSynchronize(C->side2));
  GDSW_HIP(hipStreamSynchronize(s));
  GDSW_HIP(hipStreamSynchronize(C->up));
  C->release_pinned();
  {
    unsigned long long saved = 0;
    GDSW_HIP(hipMemcpy(&saved, saved3, sizeof(saved), hipMemcpyDeviceToHost));
    const int64_t nnz1 = C->levels.empty() ? 0 : C->levels[0].K.nnz;
    st.spmv_bytes = 12.0 * (double)nnz1 - 4.0 * (double)saved + 24.0 * (double)p->n;
  }
  for (void* p : C->setup_scratch) C->arena.free_one(p);
  C->setup_scratch.clear();
  for (const Level& L : C->levels) {
    check_info(L.info, L.nparts, "local block", L.index, s);
    if (L.has_coarse) {
      check_info(L.iinfo, L.nparts, "interior block", L.index, s);
      int hb = 0;
      GDSW_HIP(hipMemcpy(&hb, L.bad, sizeof(int), hipMemcpyDeviceToHost));
      if (hb)
        throw Error(GDSW_EINVAL, "level " + std::to_string(L.index) +
                                     ": K couples dofs that share no element (not an element-assembled operator)");
    }
  }
  if (coarsest) {
    int hinfo = 0;
    GDSW_HIP(hipMemcpy(&hinfo, cinfo, sizeof(int), hipMemcpyDeviceToHost));
    C->arena.free_one(dense);
    if (hinfo != 0)
      throw Error(GDSW_ESINGULAR, "coarsest operator (order " + std::to_string(K.n) + ") has a zero pivot at column " +
                                      std::to_string(hinfo - 1));
  }
  auto span = [&](int a, int b) {
    float ms = 0;
    GDSW_HIP(hipEventElapsedTime(&ms, evs[a], evs[b]));
    return (double)ms;
  };
  for (auto& pr : ev_factor) st.ms_factor += span(pr.first, pr.second);
  for (auto& pr : ev_basis) st.ms_basis += span(pr.first, pr.second);
  if (coarsest) st.ms_coarse = span(ec0, ec1);
  for (size_t l = 0; l < ev_factor.size() && l < 8; ++l) {
    st.tl_factor[l][0] = span(e_setup, ev_factor[l].first);
    st.tl_factor[l][1] = span(e_setup, ev_factor[l].second);
  }
  for (size_t l = 0; l < ev_basis.size() && l < 8; ++l) {
    st.tl_basis[l][0] = span(e_setup, ev_basis[l].first);
    st.tl_basis[l][1] = span(e_setup, ev_basis[l].second);
  }
  if (coarsest) {
    st.tl_coarsest[0] = span(e_setup, ec0);
    st.tl_coarsest[1] = span(e_setup, ec1);
  }
  for (hipEvent_t e : evs) (void)hipEventDestroy(e);
  for (size_t l = 0; l < C->levels.size(); ++l) {
    Level& L = C->levels[l];
    if (L.lu_ev[0] && L.lu_ev[1] && l < 8) {
      float ms = 0;
      GDSW_HIP(hipEventElapsedTime(&ms, L.lu_ev[0], L.lu_ev[1]));
      st.ms_lu[l] = ms;
    }
    for (hipEvent_t& e : L.lu_ev)
      if (e) {
        (void)hipEventDestroy(e);
        e = nullptr;
      }
  }
  // algorithmic bytes of one local-solve launch (the factor tiles the substitution reads, from the
  // tile masks, and 20 bytes per row) and of one apply: local factor tiles and their gathers/stores
  // on every Schwarz level, Phi_I read twice (restriction, prolongation), the coarsest dense inverse
  {
    double ab = 0;
    for (size_t l = 0; l < C->levels.size(); ++l) {
      const Level& L = C->levels[l];
      unsigned long long kept = 0;
      GDSW_HIP(hipMemcpy(&kept, L.tkept, sizeof(kept), hipMemcpyDeviceToHost));
      double rows = 0;
      for (int d : L.dims) rows += d;
      const double bytes = (double)kept * sizeof(T) + 20.0 * rows;
      if (l < 8) st.local_solve_bytes_level[l] = bytes;
      if (l == 0) st.local_solve_bytes = bytes;
      ab += (double)kept * sizeof(T) + 24.0 * rows;
      if (L.has_coarse) ab += 2.0 * (double)L.phi_elems * sizeof(T);
    }
    if (coarsest) ab += 8.0 * (double)C->nc * C->nc;
    st.apply_bytes = ab;
  }
  st.ms_maps = host_ms;
  st.ms_total = now_ms() - t0;
}

hipEvent_t next_event(gdsw_ctx* C) {
  if (C->ev_used == C->ev_pool.size()) {
    hipEvent_t e;
    GDSW_HIP(hipEventCreate(&e));
    C->ev_pool.push_back(e);
  }
  return C->ev_pool[C->ev_used++];
}

// Sum the recorded launch durations into the statistics and recycle the events.
void drain_events(gdsw_ctx* C) {
  for (size_t k = 0; k + 1 < C->ev_used; k += 2) {
    GDSW_HIP(hipEventSynchronize(C->ev_pool[k + 1]));
    float ms = 0;
    GDSW_HIP(hipEventElapsedTime(&ms, C->ev_pool[k], C->ev_pool[k + 1]));
    const int l = C->ev_level[k / 2];
    if (l == 0) {
      C->stats.ms_local_solve += ms;
      C->stats.local_solve_launches++;
    }
    if (l < 8) {
      C->stats.ms_local_solve_level[l] += ms;
      C->stats.local_solve_launches_level[l]++;
    }
  }
  C->ev_used = 0;
  C->ev_level.clear();
}

// Autotuner: for every level, time the local solves with 2, 4 and 8 wavefronts
// per matrix (two runs each on a zero right-hand side) and keep the fastest;
// a batch shape already tuned in this process (or in the cache file) reuses
// its choice.
template <typename T>
void tune_local_solves(gdsw_ctx* C, hipStream_t s) {
  hipEvent_t e0, e1;
  GDSW_HIP(hipEventCreate(&e0));
  GDSW_HIP(hipEventCreate(&e1));
  for (size_t l = 0; l < C->levels.size(); ++l) {
    Level& L = C->levels[l];
    const std::string key = tune_key("ls", (int)sizeof(T), L.index, L.nparts, L.sum_n, L.max_n);
    int cached = 0;
    if (tune_lookup(key, &cached)) {
      L.ls_waves = cached;
      if (l < 8) C->stats.ls_waves[l] = cached;
      continue;
    }
    double* r0 = C->arena.alloc_n<double>((size_t)L.n);
    GDSW_HIP(hipMemsetAsync(r0, 0, (size_t)L.n * sizeof(double), s));
    float best = 1e30f;
    int best_w = L.ls_waves;
    for (int wv : {2, 4, 8}) {
      for (int rep = 0; rep < 2; ++rep) {
        GDSW_HIP(hipEventRecord(e0, s));
        local_solves<T>(L.nparts, L.max_n, L.order, L.dom_ptr, L.gidx, L.blk_off, static_cast<const T*>(L.blocks),
                        L.pad, L.tmask_off, L.tmask, r0, L.w, l == 0, wv, s);
        GDSW_HIP(hipEventRecord(e1, s));
        GDSW_HIP(hipEventSynchronize(e1));
        float ms = 0;
        GDSW_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (rep == 1 && ms < best) {
          best = ms;
          best_w = wv;
        }
      }
    }
    L.ls_waves = best_w;
    if (l < 8) C->stats.ls_waves[l] = best_w;
    GDSW_HIP(hipStreamSynchronize(s));   // r0 goes back to the block cache
    C->arena.free_one(r0);
    tune_store(key, best_w);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

template <typename T>
void apply_level(gdsw_ctx* C, int l, const double* r, double* z, hipStream_t s);

// Coarse correction of level l: Phi^T r, the next level (or the coarsest solve), then L.yc.
template <typename T>
void coarse_chain(gdsw_ctx* C, int l, const double* r, hipStream_t s) {
  Level& L = C->levels[l];
  const T* phi = static_cast<const T*>(L.phi);
  restrict_phi<T>(L.n_coarse, L.col_ptr, L.col_dofs, L.cp_ptr, L.cp_part, L.cp_lc, L.int_ptr, L.inter, L.phi_off, phi,
                  r, L.rc, s);
  if (l + 1 < (int)C->levels.size()) apply_level<T>(C, l + 1, L.rc, L.yc, s);
  else dense_gemv_rows(C->nc, C->ainv, L.rc, L.yc, s);
}

// z = B_l r (eq. (2.2) from level l down).  On levels 1 and 2 (level 1 only in
// captured graphs) the coarse chain runs on a side stream concurrently with the
// local solves; both join before z += Phi y.
template <typename T>
void apply_level(gdsw_ctx* C, int l, const double* r, double* z, hipStream_t s) {
  Level& L = C->levels[l];
  hipStream_t fs = (l == 0) ? C->side : (l == 1) ? C->side2 : nullptr;
  hipEvent_t ev_fork = (l == 0) ? C->ev_fork : C->ev_fork2, ev_join = (l == 0) ? C->ev_join : C->ev_join2;
  // (inside a graph capture only level 1 forks: a nested fork during capture
  // is not used)
  const bool fork = L.has_coarse && fs != nullptr && ev_fork != nullptr && (l == 0 || !C->capturing);
  if (fork) {
    GDSW_HIP(hipEventRecord(ev_fork, s));
    GDSW_HIP(hipStreamWaitEvent(fs, ev_fork, 0));
    coarse_chain<T>(C, l, r, fs);
    GDSW_HIP(hipEventRecord(ev_join, fs));
  }
  const bool prof = C->opt.profile && !C->capturing && !C->no_alloc_call;
  hipEvent_t e_start = nullptr, e_stop = nullptr;
  if (prof) {
    if (C->ev_used + 2 > 4096) drain_events(C);
    e_start = next_event(C);
    e_stop = next_event(C);
    C->ev_level.push_back(l);
  }
  local_solves<T>(L.nparts, L.max_n, L.order, L.dom_ptr, L.gidx, L.blk_off, static_cast<const T*>(L.blocks), L.pad,
                  L.tmask_off, L.tmask, r, L.w, l == 0, L.ls_waves, s, e_start, e_stop);
  scatter_sum(L.n, L.sc_ptr, L.sc_pos, L.w, z, s);
  if (!L.has_coarse) return;
  if (fork) GDSW_HIP(hipStreamWaitEvent(s, ev_join, 0));
  else coarse_chain<T>(C, l, r, s);
  const T* phi = static_cast<const T*>(L.phi);
  prolong_add<T>(L.nparts, L.max_m, L.n_gdofs, L.gdofs, L.dof_gcol, L.int_ptr, L.inter, L.pc_ptr, L.pcols, L.phi_off,
                 phi, L.yc, z, s);
}

void apply_any(gdsw_ctx* C, const double* r, double* z, hipStream_t s) {
  if (C->mixed) apply_level<float>(C, 0, r, z, s);
  else apply_level<double>(C, 0, r, z, s);
}

// ---- several right-hand sides ----------------------------------------------
// Z[:, s] = B_l R[:, s] for s < k: the local solves of each level stream every
// factor once per chunk of right-hand sides; everything else runs per
// right-hand side with the single-vector kernels.  Every column agrees with the
// single apply of that column to rounding (the multi-vector local solves update
// on MFMA).
void ensure_multi_level(gdsw_ctx* C, int k) {
  for (Level& L : C->levels) {
    if (L.multi_cap >= k) continue;
    L.wm = C->arena.alloc_n<double>((size_t)L.sum_n * k);
    if (L.has_coarse) {
      L.rcm = C->arena.alloc_n<double>((size_t)L.n_coarse * k);
      L.ycm = C->arena.alloc_n<double>((size_t)L.n_coarse * k);
    }
    L.multi_cap = k;
  }
}

template <typename T>
void apply_level_multi(gdsw_ctx* C, int l, const double* R, int64_t ldr, double* Z, int64_t ldz, int k,
                       hipStream_t s);

template <typename T>
void coarse_chain_multi(gdsw_ctx* C, int l, const double* R, int64_t ldr, int k, hipStream_t s) {
  Level& L = C->levels[l];
  const T* phi = static_cast<const T*>(L.phi);
  const int64_t nc = L.n_coarse;
  for (int q = 0; q < k; ++q)
    restrict_phi<T>(L.n_coarse, L.col_ptr, L.col_dofs, L.cp_ptr, L.cp_part, L.cp_lc, L.int_ptr, L.inter, L.phi_off,
                    phi, R + q * ldr, L.rcm + q * nc, s);
  if (l + 1 < (int)C->levels.size()) {
    apply_level_multi<T>(C, l + 1, L.rcm, nc, L.ycm, nc, k, s);
  } else {
    for (int q = 0; q < k; ++q) dense_gemv_rows(C->nc, C->ainv, L.rcm + q * nc, L.ycm + q * nc, s);
  }
}

template <typename T>
void apply_level_multi(gdsw_ctx* C, int l, const double* R, int64_t ldr, double* Z, int64_t ldz, int k,
                       hipStream_t s) {
  Level& L = C->levels[l];
  const bool fork = L.has_coarse && l == 0;
  if (fork) {
    GDSW_HIP(hipEventRecord(C->ev_fork, s));
    GDSW_HIP(hipStreamWaitEvent(C->side, C->ev_fork, 0));
    coarse_chain_multi<T>(C, l, R, ldr, k, C->side);
    GDSW_HIP(hipEventRecord(C->ev_join, C->side));
  }
  local_solves_multi<T>(L.nparts, L.max_n, L.order, L.dom_ptr, L.gidx, L.blk_off, static_cast<const T*>(L.blocks),
                        L.pad, L.tmask_off, L.tmask, R, ldr, L.wm, L.sum_n, k, s);
  for (int q = 0; q < k; ++q) scatter_sum(L.n, L.sc_ptr, L.sc_pos, L.wm + q * L.sum_n, Z + q * ldz, s);
  if (!L.has_coarse) return;
  if (fork) GDSW_HIP(hipStreamWaitEvent(s, C->ev_join, 0));
  else coarse_chain_multi<T>(C, l, R, ldr, k, s);
  const T* phi = static_cast<const T*>(L.phi);
  const int64_t nc = L.n_coarse;
  for (int q = 0; q < k; ++q)
    prolong_add<T>(L.nparts, L.max_m, L.n_gdofs, L.gdofs, L.dof_gcol, L.int_ptr, L.inter, L.pc_ptr, L.pcols,
                   L.phi_off, phi, L.ycm + q * nc, Z + q * ldz, s);
}

void apply_multi_any(gdsw_ctx* C, const double* R, int64_t ldr, double* Z, int64_t ldz, int k, hipStream_t s) {
  ensure_multi_level(C, k);
  if (C->mixed) apply_level_multi<float>(C, 0, R, ldr, Z, ldz, k, s);
  else apply_level_multi<double>(C, 0, R, ldr, Z, ldz, k, s);
}

// Device workspace of one FGMRES(m) solve on n rows.
struct KrylovWs {
  double *V = nullptr, *Z = nullptr, *w = nullptr, *dpart = nullptr, *hdev = nullptr, *ydev = nullptr;
};

// Sizes (doubles) of the workspace pieces, in the order V, Z, w, dpart, hdev, ydev.
std::array<size_t, 6> krylov_ws_sizes(int64_t n, int m) {
  return {(size_t)n * (m + 1), (size_t)n * m, (size_t)n, (size_t)multi_dot_blocks(n) * (m + 2),
          (size_t)2 * (m + 2) + 2, (size_t)m + 1};
}

// Carve the pieces out of one region; every piece starts on a 256-byte boundary.
// Returns the doubles used (base == nullptr: only the size).
size_t carve_krylov_ws(double* base, int64_t n, int m, KrylovWs* ws) {
  const std::array<size_t, 6> sz = krylov_ws_sizes(n, m);
  double** dst[6] = {&ws->V, &ws->Z, &ws->w, &ws->dpart, &ws->hdev, &ws->ydev};
  size_t off = 0;
  for (int k = 0; k < 6; ++k) {
    if (base) *dst[k] = base + off;
    off += (sz[k] + 31) & ~size_t(31);
  }
  return off;
}

// Host-side resources every solve needs, created at setup (the page-locked
// buffer the Hessenberg column is read into, its event, the Givens arrays).
void create_solve_host_state(gdsw_ctx* C) {
  const int m = C->opt.restart;
  if (!C->hhost) GDSW_HIP(hipHostMalloc((void**)&C->hhost, sizeof(double) * (2 * 256 + 8), hipHostMallocDefault));
  if (!C->ev_fetch) GDSW_HIP(hipEventCreateWithFlags(&C->ev_fetch, hipEventDisableTiming));
  C->kH.assign((size_t)(m + 1) * m, 0.0);
  C->kcs.assign(m, 0.0);
  C->ksn.assign(m, 0.0);
  C->kg.assign(m + 1, 0.0);
  C->ky.assign(m, 0.0);
}

// The context's own workspace, allocated on its first solve.
KrylovWs context_workspace(gdsw_ctx* C) {
  const int m = C->opt.restart;
  if (C->ws_m != m) {
    const int64_t n = C->levels[0].n;
    const std::array<size_t, 6> sz = krylov_ws_sizes(n, m);
    Arena& A = C->arena;
    C->V = A.alloc_n<double>(sz[0]);
    C->Z = A.alloc_n<double>(sz[1]);
    C->wv = A.alloc_n<double>(sz[2]);
    C->dpart = A.alloc_n<double>(sz[3]);
    C->hdev = A.alloc_n<double>(sz[4]);
    C->ydev = A.alloc_n<double>(sz[5]);
    C->ws_m = m;
  }
  KrylovWs ws;
  ws.V = C->V;
  ws.Z = C->Z;
  ws.w = C->wv;
  ws.dpart = C->dpart;
  ws.hdev = C->hdev;
  ws.ydev = C->ydev;
  return ws;
}

// Apply of Krylov column j: eager, or replay of the graph captured for that column.
void column_apply(gdsw_ctx* C, int j, const double* v, double* z, hipStream_t s) {
  if (!C->opt.graph || C->no_alloc_call) {
    apply_any(C, v, z, s);
    return;
  }
  if ((int)C->apply_exec.size() <= j) C->apply_exec.resize(j + 1, nullptr);
  if (!C->apply_exec[j]) {
    hipGraph_t g = nullptr;
    C->capturing = true;
    GDSW_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      apply_any(C, v, z, s);
    } catch (...) {
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
      C->capturing = false;
      throw;
    }
    GDSW_HIP(hipStreamEndCapture(s, &g));
    C->capturing = false;
    hipGraphExec_t exec = nullptr;
    GDSW_HIP(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    C->apply_exec[j] = exec;
  }
  GDSW_HIP(hipGraphLaunch(C->apply_exec[j], s));
}

// FGMRES(m) on the workspace ws.  use_graph: applies replay captured graphs
// (graph = 1 contexts, gdsw_solve only).  precond: another preconditioner in
// place of the context's apply (the multigrid cycle).
using Precond = std::function<void(const double*, double*, hipStream_t)>;

int solve_impl(gdsw_ctx* C, const double* b, double* x, hipStream_t caller, gdsw_solve_info* info,
               const KrylovWs& ws, bool use_graph, const Precond* precond = nullptr) {
  const double t0 = now_ms();
  hipStream_t s = caller;
  if (use_graph) {               // captured work needs a stream of its own (not the legacy default stream)
    if (!C->own) {
      GDSW_HIP(hipStreamCreateWithFlags(&C->own, hipStreamNonBlocking));
      GDSW_HIP(hipEventCreateWithFlags(&C->ev_in, hipEventDisableTiming));
      GDSW_HIP(hipEventCreateWithFlags(&C->ev_out, hipEventDisableTiming));
    }
    GDSW_HIP(hipEventRecord(C->ev_in, caller));
    GDSW_HIP(hipStreamWaitEvent(C->own, C->ev_in, 0));
    s = C->own;
  }
  struct Rejoin {
    gdsw_ctx* C;
    hipStream_t caller;
    bool on;
    ~Rejoin() {
      if (on && C->own) {
        (void)hipEventRecord(C->ev_out, C->own);
        (void)hipStreamWaitEvent(caller, C->ev_out, 0);
      }
    }
  } rejoin{C, caller, use_graph};
  const int m = C->opt.restart;
  const int64_t n = C->levels[0].n;
  const CsrDev& K = C->levels[0].K;
  double* V = ws.V;
  double* Z = ws.Z;
  double* w = ws.w;
  double* dpart = ws.dpart;
  double* h1 = ws.hdev;               // [m+1]
  double* h2 = ws.hdev + (m + 1);     // [m+1]
  double* nr = ws.hdev + 2 * (m + 1); // [1]
  double* gate = nr + 1;              // [1] second Gram-Schmidt pass taken
  double* hh = C->hhost;
  // the host polls an event after the copy (lower wake-up latency than a
  // blocking stream synchronization; the Krylov loop waits here every step)
  auto fetch = [&](int count) {
    GDSW_HIP(hipMemcpyAsync(hh, ws.hdev, count * sizeof(double), hipMemcpyDeviceToHost, s));
    GDSW_HIP(hipEventRecord(C->ev_fetch, s));
    wait_event_polling(C->ev_fetch);
  };
  multi_dot(n, 1, b, n, b, dpart, nr, s);
  GDSW_HIP(hipMemcpyAsync(hh, nr, sizeof(double), hipMemcpyDeviceToHost, s));
  GDSW_HIP(hipStreamSynchronize(s));
  const double bnorm = std::sqrt(hh[0]);
  GDSW_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s));
  gdsw_solve_info inf;
  std::memset(&inf, 0, sizeof(inf));
  if (bnorm == 0.0) {
    inf.converged = 1;
    if (info) *info = inf;
    return GDSW_OK;
  }
  std::vector<double>& H = C->kH;
  std::vector<double>& cs = C->kcs;
  std::vector<double>& sn = C->ksn;
  std::vector<double>& g = C->kg;
  std::vector<double>& y = C->ky;
  int its = 0;
  double ms_apply = 0, ms_spmv = 0, ms_orth = 0;
  const bool timing = std::getenv("GDSW_PHASE_TIMING") != nullptr;
  auto tick = [&](double& acc, double& last) {
    if (!timing) return;
    GDSW_HIP(hipStreamSynchronize(s));
    const double t = now_ms();
    acc += t - last;
    last = t;
  };
  while (true) {
    spmv(K, x, V, s);
    residual_from(n, b, V, s);
    multi_dot(n, 1, V, n, V, dpart, nr, s);
    GDSW_HIP(hipMemcpyAsync(hh, nr, sizeof(double), hipMemcpyDeviceToHost, s));
    GDSW_HIP(hipStreamSynchronize(s));
    const double beta = std::sqrt(hh[0]);
    inf.rel_residual = beta / bnorm;
    if (inf.rel_residual <= C->opt.tol) {
      inf.converged = 1;
      break;
    }
    if (its >= C->opt.max_it) break;
    scale_by_inv_norm(n, V, nr, V, s);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      double last = now_ms(), dummy = 0;
      if (timing) {
        GDSW_HIP(hipStreamSynchronize(s));
        last = now_ms();
      }
      double* vj = V + (int64_t)j * n;
      double* zj = Z + (int64_t)j * n;
      if (precond) (*precond)(vj, zj, s);
      else column_apply(C, j, vj, zj, s);
      tick(ms_apply, last);
      spmv(K, zj, w, s);
      tick(ms_spmv, last);
      // classical Gram-Schmidt, reorthogonalised where needed
      gram_schmidt(n, j + 1, V, n, w, dpart, h1, h2, nr, gate, s);
      scale_by_inv_norm(n, w, nr, V + (int64_t)(j + 1) * n, s);
      fetch(2 * (m + 1) + 2);
      tick(ms_orth, last);
      (void)dummy;
      double* Hj = H.data() + (size_t)j * (m + 1);
      for (int i = 0; i <= j; ++i) Hj[i] = hh[i] + hh[(m + 1) + i];
      Hj[j + 1] = std::sqrt(hh[2 * (m + 1)]);
      if (hh[2 * (m + 1) + 1] > 0.5) inf.reorthogonalizations++;
      const bool breakdown = Hj[j + 1] == 0.0;
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
        Hj[i + 1] = -sn[i] * Hj[i] + cs[i] * Hj[i + 1];
        Hj[i] = t;
      }
      const double den = std::hypot(Hj[j], Hj[j + 1]);
      cs[j] = den > 0 ? Hj[j] / den : 1.0;
      sn[j] = den > 0 ? Hj[j + 1] / den : 0.0;
      Hj[j] = den;
      Hj[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      k = j + 1;
      if (std::fabs(g[j + 1]) / bnorm <= C->opt.tol || its >= C->opt.max_it || breakdown) break;
    }
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int q = i + 1; q < k; ++q) t -= H[(size_t)q * (m + 1) + i] * y[q];
      const double d = H[(size_t)i * (m + 1) + i];
      y[i] = d != 0.0 ? t / d : 0.0;
    }
    for (int i = 0; i < k; ++i) hh[i] = -y[i];
    GDSW_HIP(hipMemcpyAsync(ws.ydev, hh, k * sizeof(double), hipMemcpyHostToDevice, s));
    multi_axpy(n, k, Z, n, ws.ydev, x, s);
    GDSW_HIP(hipStreamSynchronize(s));   // the host buffer is reused by the next fetch
    inf.restarts++;
  }
  inf.iterations = its;
  inf.ms_apply = ms_apply;
  inf.ms_spmv = ms_spmv;
  inf.ms_orth = ms_orth;
  inf.ms_total = now_ms() - t0;
  if (info) *info = inf;
  return inf.converged ? GDSW_OK : GDSW_NOTCONV;
}

// k FGMRES(m) solves in lockstep on one context: every inner iteration applies
// the preconditioner to the current Krylov vectors of all k systems at once
// (one pass over the local factors per chunk of systems); SpMV, Gram-Schmidt,
// Givens rotations, restarts and convergence are those of solve_impl, per
// system, so each x_s follows gdsw_solve's iteration for b_s (to rounding).  A system that
// has converged (or reached max_it) keeps its iterate; its columns of the
// shared apply are computed and ignored.
int solve_multi_impl(gdsw_ctx* C, int k, const double* B, int64_t ldb, double* X, int64_t ldx, hipStream_t s,
                     gdsw_solve_info* infos) {
  const double t0 = now_ms();
  const int m = C->opt.restart;
  const int64_t n = C->levels[0].n;
  const CsrDev& K = C->levels[0].K;
  const int hs = 2 * (m + 1) + 2;             // per-system slots (h1, h2, norm, second-pass flag)
  if (C->multi_cap < k || C->multi_m != m) {
    Arena& A = C->arena;
    C->mV = A.alloc_n<double>((size_t)k * n * (m + 1));
    C->mZ = A.alloc_n<double>((size_t)k * n * m);
    C->mW = A.alloc_n<double>((size_t)k * n);
    C->mH = A.alloc_n<double>((size_t)k * hs);
    C->mY = A.alloc_n<double>((size_t)k * (m + 1));
    C->mP = A.alloc_n<double>((size_t)multi_dot_blocks(n) * (m + 2));
    if (C->mhost) (void)hipHostFree(C->mhost);
    C->mhost = nullptr;
    GDSW_HIP(hipHostMalloc((void**)&C->mhost, sizeof(double) * ((size_t)k * hs + (size_t)k * (m + 1) + 8),
                           hipHostMallocDefault));
    C->multi_cap = k;
    C->multi_m = m;
  }
  const int64_t ldv = n * (m + 1), ldzz = n * m;
  double* hh = C->mhost;
  double* hy = C->mhost + (size_t)k * hs;
  auto Vs = [&](int q) { return C->mV + q * ldv; };
  auto Zs = [&](int q) { return C->mZ + q * ldzz; };
  auto Hs = [&](int q) { return C->mH + (int64_t)q * hs; };
  auto fetch_all = [&]() {
    GDSW_HIP(hipMemcpyAsync(hh, C->mH, (size_t)k * hs * sizeof(double), hipMemcpyDeviceToHost, s));
    GDSW_HIP(hipEventRecord(C->ev_fetch, s));
    wait_event_polling(C->ev_fetch);
  };
  struct Sys {
    double bnorm = 0, beta = 0;
    int its = 0, k = 0, restarts = 0, reorth = 0;
    bool done = false, conv = false, running = false;
    std::vector<double> H, cs, sn, g, y;
  };
  std::vector<Sys> sy(k);
  for (int q = 0; q < k; ++q) {
    Sys& S = sy[q];
    S.H.assign((size_t)(m + 1) * m, 0.0);
    S.cs.assign(m, 0.0);
    S.sn.assign(m, 0.0);
    S.g.assign(m + 1, 0.0);
    S.y.assign(m, 0.0);
    multi_dot(n, 1, B + q * ldb, n, B + q * ldb, C->mP, Hs(q) + 2 * (m + 1), s);
    GDSW_HIP(hipMemsetAsync(X + q * ldx, 0, n * sizeof(double), s));
  }
  fetch_all();
  for (int q = 0; q < k; ++q) {
    sy[q].bnorm = std::sqrt(hh[(size_t)q * hs + 2 * (m + 1)]);
    if (sy[q].bnorm == 0.0) {
      sy[q].done = true;
      sy[q].conv = true;
    }
  }
  std::vector<double> rel(k, 0.0);
  while (true) {
    // true residuals of the systems still going
    bool any = false;
    for (int q = 0; q < k; ++q) {
      if (sy[q].done) continue;
      spmv(K, X + q * ldx, Vs(q), s);
      residual_from(n, B + q * ldb, Vs(q), s);
      multi_dot(n, 1, Vs(q), n, Vs(q), C->mP, Hs(q) + 2 * (m + 1), s);
      any = true;
    }
    if (!any) break;
    fetch_all();
    bool cycle = false;
    for (int q = 0; q < k; ++q) {
      Sys& S = sy[q];
      S.running = false;
      if (S.done) continue;
      S.beta = std::sqrt(hh[(size_t)q * hs + 2 * (m + 1)]);
      rel[q] = S.beta / S.bnorm;
      if (rel[q] <= C->opt.tol) {
        S.done = S.conv = true;
        continue;
      }
      if (S.its >= C->opt.max_it) {
        S.done = true;
        continue;
      }
      scale_by_inv_norm(n, Vs(q), Hs(q) + 2 * (m + 1), Vs(q), s);
      std::fill(S.H.begin(), S.H.end(), 0.0);
      std::fill(S.g.begin(), S.g.end(), 0.0);
      S.g[0] = S.beta;
      S.k = 0;
      S.running = true;
      cycle = true;
    }
    if (!cycle) break;          // every remaining system converged or stopped at this check
    for (int j = 0; j < m; ++j) {
      bool run = false;
      for (const Sys& S : sy) run |= S.running;
      if (!run) break;
      // the preconditioner on column j of every system (stride n (m + 1) between systems)
      apply_multi_any(C, C->mV + (int64_t)j * n, ldv, C->mZ + (int64_t)j * n, ldzz, k, s);
      for (int q = 0; q < k; ++q) {
        if (!sy[q].running) continue;
        double* V = Vs(q);
        double* zj = Zs(q) + (int64_t)j * n;
        double* w = C->mW + q * n;
        double* h1 = Hs(q);
        double* h2 = Hs(q) + (m + 1);
        double* nr = Hs(q) + 2 * (m + 1);
        spmv(K, zj, w, s);
        gram_schmidt(n, j + 1, V, n, w, C->mP, h1, h2, nr, nr + 1, s);
        scale_by_inv_norm(n, w, nr, V + (int64_t)(j + 1) * n, s);
      }
      fetch_all();
      for (int q = 0; q < k; ++q) {
        Sys& S = sy[q];
        if (!S.running) continue;
        const double* hq = hh + (size_t)q * hs;
        double* Hj = S.H.data() + (size_t)j * (m + 1);
        for (int i = 0; i <= j; ++i) Hj[i] = hq[i] + hq[(m + 1) + i];
        Hj[j + 1] = std::sqrt(hq[2 * (m + 1)]);
        if (hq[2 * (m + 1) + 1] > 0.5) S.reorth++;
        const bool breakdown = Hj[j + 1] == 0.0;
        for (int i = 0; i < j; ++i) {
          const double t = S.cs[i] * Hj[i] + S.sn[i] * Hj[i + 1];
          Hj[i + 1] = -S.sn[i] * Hj[i] + S.cs[i] * Hj[i + 1];
          Hj[i] = t;
        }
        const double den = std::hypot(Hj[j], Hj[j + 1]);
        S.cs[j] = den > 0 ? Hj[j] / den : 1.0;
        S.sn[j] = den > 0 ? Hj[j + 1] / den : 0.0;
        Hj[j] = den;
        Hj[j + 1] = 0.0;
        S.g[j + 1] = -S.sn[j] * S.g[j];
        S.g[j] = S.cs[j] * S.g[j];
        ++S.its;
        S.k = j + 1;
        if (std::fabs(S.g[j + 1]) / S.bnorm <= C->opt.tol || S.its >= C->opt.max_it || breakdown) S.running = false;
      }
    }
    // x += Z y for every system of this cycle
    for (int q = 0; q < k; ++q) {
      Sys& S = sy[q];
      if (S.done || S.k == 0) continue;
      const int kq = S.k;
      for (int i = kq - 1; i >= 0; --i) {
        double t = S.g[i];
        for (int c = i + 1; c < kq; ++c) t -= S.H[(size_t)c * (m + 1) + i] * S.y[c];
        const double d = S.H[(size_t)i * (m + 1) + i];
        S.y[i] = d != 0.0 ? t / d : 0.0;
      }
      for (int i = 0; i < kq; ++i) hy[(size_t)q * (m + 1) + i] = -S.y[i];
      GDSW_HIP(hipMemcpyAsync(C->mY + (int64_t)q * (m + 1), hy + (size_t)q * (m + 1), kq * sizeof(double),
                              hipMemcpyHostToDevice, s));
      multi_axpy(n, kq, Zs(q), n, C->mY + (int64_t)q * (m + 1), X + q * ldx, s);
      S.restarts++;
      S.k = 0;
    }
    GDSW_HIP(hipStreamSynchronize(s));   // the host buffers are reused by the next fetch
  }
  int code = GDSW_OK;
  const double total = now_ms() - t0;
  for (int q = 0; q < k; ++q) {
    gdsw_solve_info inf;
    std::memset(&inf, 0, sizeof(inf));
    inf.iterations = sy[q].its;
    inf.restarts = sy[q].restarts;
    inf.reorthogonalizations = sy[q].reorth;
    inf.converged = sy[q].conv ? 1 : 0;
    inf.rel_residual = rel[q];
    inf.ms_total = total;
    if (infos) infos[q] = inf;
    if (!sy[q].conv) code = GDSW_NOTCONV;
  }
  return code;
}

int fail(const Error& e) {
  g_last_error = e.what();
  return e.code;
}

}  // namespace
}  // namespace gdsw

// Two-grid geometric multigrid whose coarse problem is solved by FGMRES
// preconditioned by a GDSW hierarchy (section 3, second role): the fine
// operator and the smoother come from a one-level context on the fine problem,
// the coarse solver from a context on the coarse problem (its tol is the
// coarse reduction), P / P^T are the grid transfers.
struct gdsw_mg {
  gdsw_ctx* fine = nullptr;
  gdsw_ctx* coarse = nullptr;
  gdsw::Arena arena;
  gdsw::CsrDev P, PT;
  double *d = nullptr, *t = nullptr, *dc = nullptr, *ec = nullptr;
  int nu_pre = 2, nu_post = 2;
  double omega = 1.0;
  int64_t cycles = 0, coarse_its = 0;
  std::map<hipStream_t, hipEvent_t> stream_marks;
  ~gdsw_mg() {
    for (auto& kv : stream_marks) {
      (void)hipEventSynchronize(kv.second);
      (void)hipEventDestroy(kv.second);
    }
  }
};

namespace gdsw {
namespace {

CsrDev copy_csr(Arena& A, int64_t rows, const int64_t* rowptr, const int* col, const double* val, hipStream_t s) {
  int64_t nnz = 0;
  GDSW_HIP(hipMemcpyAsync(&nnz, rowptr + rows, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  GDSW_HIP(hipStreamSynchronize(s));
  if (nnz < 0) throw Error(GDSW_EINVAL, "negative nonzero count");
  CsrDev M;
  M.n = rows;
  M.nnz = nnz;
  int64_t* rp = A.alloc_n<int64_t>(rows + 1);
  int* cl = A.alloc_n<int>((size_t)std::max<int64_t>(nnz, 1));
  double* vl = A.alloc_n<double>((size_t)std::max<int64_t>(nnz, 1));
  GDSW_HIP(hipMemcpyAsync(rp, rowptr, (rows + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  if (nnz) {
    GDSW_HIP(hipMemcpyAsync(cl, col, nnz * sizeof(int), hipMemcpyDeviceToDevice, s));
    GDSW_HIP(hipMemcpyAsync(vl, val, nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  M.rowptr = rp;
  M.col = cl;
  M.val = vl;
  return M;
}

// One cycle z = M r (z starts at 0): pre-smoothing, coarse-grid correction by the inexact
// coarse solve, post-smoothing; every step in the oracle's order.
void mg_cycle(gdsw_mg* M, const double* r, double* z, hipStream_t s) {
  const CsrDev& Kf = M->fine->levels[0].K;
  const int64_t n = Kf.n;
  auto smooth = [&](bool first) {
    if (first) {
      apply_any(M->fine, r, M->t, s);                 // S (r - K 0)
      axpby(n, M->omega, M->t, 0.0, z, s);
    } else {
      spmv(Kf, z, M->d, s);
      residual_from(n, r, M->d, s);
      apply_any(M->fine, M->d, M->t, s);
      axpby(n, M->omega, M->t, 1.0, z, s);
    }
  };
  for (int k = 0; k < M->nu_pre; ++k) smooth(k == 0);
  const double* d = r;
  if (M->nu_pre > 0) {
    spmv(Kf, z, M->d, s);
    residual_from(n, r, M->d, s);
    d = M->d;
  }
  spmv(M->PT, d, M->dc, s);
  gdsw_solve_info inf;
  const KrylovWs ws = context_workspace(M->coarse);
  solve_impl(M->coarse, M->dc, M->ec, s, &inf, ws, false);
  M->coarse_its += inf.iterations;
  M->cycles++;
  spmv(M->P, M->ec, M->t, s);
  if (M->nu_pre > 0) axpby(n, 1.0, M->t, 1.0, z, s);
  else axpby(n, 1.0, M->t, 0.0, z, s);
  for (int k = 0; k < M->nu_post; ++k) smooth(false);
}

// A setup that fails part way may already have queued kernels on the caller's
// stream that write blocks of the context's arena.  Those blocks go back to the
// process-wide cache when the context is deleted, where a concurrent setup on
// another stream could take them, so the caller's stream is drained first (the
// context's own streams are drained by its destructor).  The message of the
// original failure is kept.
void discard_failed_setup(gdsw_ctx* C, hipStream_t s) {
  const std::string msg = g_last_error;
  (void)hipStreamSynchronize(s);
  delete C;
  g_last_error = msg;
}

}  // namespace
}  // namespace gdsw

// Krylov workspace of gdsw_solve_noalloc: a static device array (one copy per
// device the library runs on, held until the process ends).  Host code never
// uses its name as a device address: the address is looked up once per device
// with hipGetSymbolAddress and kept in scratch_dev.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace gdsw {
namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_dev[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first call
// on that device, with that device current).
double* scratch_on_current_device() {
  int dev = 0;
  GDSW_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) throw Error(GDSW_EINVAL, "device id out of range");
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    GDSW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    scratch_dev[dev] = static_cast<double*>(p);
  }
  return scratch_dev[dev];
}
}  // namespace
}  // namespace gdsw

using gdsw::Error;

namespace gdsw {
namespace {
// Records (creating on first use) the mark event of stream s in `marks` when the guard goes out
// of scope, also when the call throws.
struct StreamMark {
  std::map<hipStream_t, hipEvent_t>* marks;
  hipStream_t s;
  ~StreamMark() {
    if (!marks) return;
    hipEvent_t& e = (*marks)[s];
    if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      e = nullptr;
      return;
    }
    (void)hipEventRecord(e, s);
  }
};
}  // namespace
}  // namespace gdsw

extern "C" {

void gdsw_default_options(gdsw_options* o) {
  if (!o) return;
  o->overlap = 1;
  o->combine = GDSW_COMBINE_RESTRICTED;
  o->precision = GDSW_FP64;
  o->restart = 30;
  o->max_it = 1000;
  o->tol = 1e-8;
  o->no_coarse = 0;
  o->panel = 0;
  o->profile = 0;
  o->graph = 0;
  o->tune = 0;
  o->ls_waves = 0;
  o->lu_variant = 0;
  o->pressure_gamma = 0;
}

const char* gdsw_last_error(void) { return gdsw::g_last_error.c_str(); }

int gdsw_setup(const gdsw_problem* prob, const gdsw_options* opt, void* stream, gdsw_ctx** out) {
  if (!out) {
    gdsw::g_last_error = "out is NULL";
    return GDSW_EINVAL;
  }
  *out = nullptr;
  gdsw_ctx* C = new (std::nothrow) gdsw_ctx();
  if (!C) {
    gdsw::g_last_error = "host allocation failed";
    return GDSW_ENOMEM;
  }
  try {
    gdsw_default_options(&C->opt);
    if (opt) C->opt = *opt;
    if (C->opt.overlap < 0 || C->opt.restart < 1 || C->opt.restart > 250 || C->opt.max_it < 0 ||
        !(C->opt.tol >= 0.0) || (C->opt.combine != 0 && C->opt.combine != 1) ||
        (C->opt.precision != 0 && C->opt.precision != 1) ||
        (C->opt.ls_waves != 0 && C->opt.ls_waves != 2 && C->opt.ls_waves != 4 && C->opt.ls_waves != 8) ||
        C->opt.tune < 0 || C->opt.tune > 3 || C->opt.lu_variant < 0 || C->opt.lu_variant > 7 ||
        (C->opt.pressure_gamma != 0 && C->opt.pressure_gamma != 1))
      throw Error(GDSW_EINVAL, "invalid options");
    C->mixed = C->opt.precision == GDSW_MIXED;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GDSW_HIP(hipStreamCreateWithFlags(&C->side, hipStreamNonBlocking));
    GDSW_HIP(hipStreamCreateWithFlags(&C->side2, hipStreamNonBlocking));
    GDSW_HIP(hipStreamCreateWithFlags(&C->up, hipStreamNonBlocking));
    GDSW_HIP(hipEventCreateWithFlags(&C->ev_up, hipEventDisableTiming));
    GDSW_HIP(hipEventCreateWithFlags(&C->ev_fork, hipEventDisableTiming));
    GDSW_HIP(hipEventCreateWithFlags(&C->ev_join, hipEventDisableTiming));
    GDSW_HIP(hipEventCreateWithFlags(&C->ev_fork2, hipEventDisableTiming));
    GDSW_HIP(hipEventCreateWithFlags(&C->ev_join2, hipEventDisableTiming));
    if (C->mixed) gdsw::setup_impl<float>(C, prob, s);
    else gdsw::setup_impl<double>(C, prob, s);
    for (size_t l = 0; l < C->levels.size() && l < 8; ++l) {
      C->stats.ls_waves[l] = C->levels[l].ls_waves;
      C->stats.lu_variant[l] = C->levels[l].lu_variant;
    }
    gdsw::create_solve_host_state(C);
    if (C->opt.tune & 1) {
      if (C->mixed) gdsw::tune_local_solves<float>(C, s);
      else gdsw::tune_local_solves<double>(C, s);
    }
    GDSW_HIP(hipStreamSynchronize(s));
  } catch (const Error& e) {
    gdsw::discard_failed_setup(C, static_cast<hipStream_t>(stream));
    return gdsw::fail(e);
  } catch (const std::bad_alloc&) {
    gdsw::discard_failed_setup(C, static_cast<hipStream_t>(stream));
    gdsw::g_last_error = "host allocation failed";
    return GDSW_ENOMEM;
  }
  *out = C;
  return GDSW_OK;
}

int gdsw_apply(gdsw_ctx* C, const double* r, double* z, void* stream) {
  if (!C || !r || !z || r == z) {
    gdsw::g_last_error = "gdsw_apply: NULL or aliased argument";
    return GDSW_EINVAL;
  }
  gdsw::StreamMark mark_{&C->stream_marks, static_cast<hipStream_t>(stream)};
  try {
    gdsw::apply_any(C, r, z, static_cast<hipStream_t>(stream));
  } catch (const Error& e) {
    return gdsw::fail(e);
  }
  return GDSW_OK;
}

int gdsw_solve(gdsw_ctx* C, const double* b, double* x, void* stream, gdsw_solve_info* info) {
  if (!C || !b || !x || b == x) {
    gdsw::g_last_error = "gdsw_solve: NULL or aliased argument";
    return GDSW_EINVAL;
  }
  gdsw::StreamMark mark_{&C->stream_marks, static_cast<hipStream_t>(stream)};
  try {
    const gdsw::KrylovWs ws = gdsw::context_workspace(C);
    return gdsw::solve_impl(C, b, x, static_cast<hipStream_t>(stream), info, ws, C->opt.graph != 0);
  } catch (const Error& e) {
    return gdsw::fail(e);
  }
}

int gdsw_solve_noalloc(gdsw_ctx* C, const double* b, double* x, void* stream, gdsw_solve_info* info) {
  if (!C || !b || !x || b == x) {
    gdsw::g_last_error = "gdsw_solve_noalloc: NULL or aliased argument";
    return GDSW_EINVAL;
  }
  gdsw::StreamMark mark_{&C->stream_marks, static_cast<hipStream_t>(stream)};
  try {
    const int64_t n = C->levels[0].n;
    const int m = C->opt.restart;
    const size_t need = gdsw::carve_krylov_ws(nullptr, n, m, nullptr) * sizeof(double);
    if (need > NOALLOC_SCRATCH_BYTES)
      throw Error(GDSW_EINVAL, "gdsw_solve_noalloc: the FGMRES workspace of n = " + std::to_string(n) +
                                   ", restart " + std::to_string(m) + " needs " + std::to_string(need) +
                                   " bytes, more than the " + std::to_string(NOALLOC_SCRATCH_BYTES) +
                                   "-byte static workspace");
    gdsw::KrylovWs ws;
    gdsw::carve_krylov_ws(gdsw::scratch_on_current_device(), n, m, &ws);
    struct Flag {
      gdsw_ctx* C;
      ~Flag() { C->no_alloc_call = false; }
    } flag{C};
    C->no_alloc_call = true;
    return gdsw::solve_impl(C, b, x, static_cast<hipStream_t>(stream), info, ws, false);
  } catch (const Error& e) {
    return gdsw::fail(e);
  }
}

int gdsw_apply_multi(gdsw_ctx* C, int32_t k, const double* R, int64_t ldr, double* Z, int64_t ldz, void* stream) {
  if (!C || !R || !Z || k < 1 || k > GDSW_MAX_RHS || ldr < C->levels[0].n || ldz < C->levels[0].n || R == Z) {
    gdsw::g_last_error = "gdsw_apply_multi: NULL, aliased or out-of-range argument";
    return GDSW_EINVAL;
  }
  gdsw::StreamMark mark_{&C->stream_marks, static_cast<hipStream_t>(stream)};
  try {
    gdsw::apply_multi_any(C, R, ldr, Z, ldz, k, static_cast<hipStream_t>(stream));
  } catch (const Error& e) {
    return gdsw::fail(e);
  }
  return GDSW_OK;
}

int gdsw_solve_multi(gdsw_ctx* C, int32_t k, const double* B, int64_t ldb, double* X, int64_t ldx, void* stream,
                     gdsw_solve_info* info) {
  if (!C || !B || !X || k < 1 || k > GDSW_MAX_RHS || ldb < C->levels[0].n || ldx < C->levels[0].n || B == X) {
    gdsw::g_last_error = "gdsw_solve_multi: NULL, aliased or out-of-range argument";
    return GDSW_EINVAL;
  }
  gdsw::StreamMark mark_{&C->stream_marks, static_cast<hipStream_t>(stream)};
  try {
    return gdsw::solve_multi_impl(C, k, B, ldb, X, ldx, static_cast<hipStream_t>(stream), info);
  } catch (const Error& e) {
    return gdsw::fail(e);
  }
}

int gdsw_mg_create(gdsw_ctx* fine, gdsw_ctx* coarse, int64_t n_fine, int64_t n_coarse, const int64_t* p_rowptr,
                   const int32_t* p_col, const double* p_val, const int64_t* pt_rowptr, const int32_t* pt_col,
                   const double* pt_val, int32_t nu_pre, int32_t nu_post, double omega, void* stream,
                   gdsw_mg** out) {
  if (!out) {
    gdsw::g_last_error = "gdsw_mg_create: out is NULL";
    return GDSW_EINVAL;
  }
  *out = nullptr;
  if (!fine || !coarse || fine == coarse || !p_rowptr || !p_col || !p_val || !pt_rowptr || !pt_col || !pt_val ||
      nu_pre < 0 || nu_post < 0 || nu_pre + nu_post > 64 || !(omega > 0.0) || fine->levels[0].n != n_fine ||
      coarse->levels[0].n != n_coarse) {
    gdsw::g_last_error = "gdsw_mg_create: NULL, inconsistent or out-of-range argument";
    return GDSW_EINVAL;
  }
  gdsw_mg* M = new (std::nothrow) gdsw_mg();
  if (!M) {
    gdsw::g_last_error = "host allocation failed";
    return GDSW_ENOMEM;
  }
  try {
    hipStream_t s = static_cast<hipStream_t>(stream);
    M->fine = fine;
    M->coarse = coarse;
    M->P = gdsw::copy_csr(M->arena, n_fine, p_rowptr, p_col, p_val, s);
    M->PT = gdsw::copy_csr(M->arena, n_coarse, pt_rowptr, pt_col, pt_val, s);
    M->d = M->arena.alloc_n<double>((size_t)n_fine);
    M->t = M->arena.alloc_n<double>((size_t)n_fine);
    M->dc = M->arena.alloc_n<double>((size_t)n_coarse);
    M->ec = M->arena.alloc_n<double>((size_t)n_coarse);
    M->nu_pre = nu_pre;
    M->nu_post = nu_post;
    M->omega = omega;
    GDSW_HIP(hipStreamSynchronize(s));
  } catch (const Error& e) {
    (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
    delete M;
    return gdsw::fail(e);
  }
  *out = M;
  return GDSW_OK;
}

int gdsw_mg_apply(gdsw_mg* M, const double* r, double* z, void* stream) {
  if (!M || !r || !z || r == z) {
    gdsw::g_last_error = "gdsw_mg_apply: NULL or aliased argument";
    return GDSW_EINVAL;
  }
  gdsw::StreamMark mark_{&M->stream_marks, static_cast<hipStream_t>(stream)};
  gdsw::StreamMark mark_f{&M->fine->stream_marks, static_cast<hipStream_t>(stream)};
  gdsw::StreamMark mark_c{&M->coarse->stream_marks, static_cast<hipStream_t>(stream)};
  try {
    gdsw::mg_cycle(M, r, z, static_cast<hipStream_t>(stream));
  } catch (const Error& e) {
    return gdsw::fail(e);
  }
  return GDSW_OK;
}

int gdsw_mg_solve(gdsw_mg* M, const double* b, double* x, void* stream, gdsw_solve_info* info) {
  if (!M || !b || !x || b == x) {
    gdsw::g_last_error = "gdsw_mg_solve: NULL or aliased argument";
    return GDSW_EINVAL;
  }
  gdsw::StreamMark mark_{&M->stream_marks, static_cast<hipStream_t>(stream)};
  gdsw::StreamMark mark_f{&M->fine->stream_marks, static_cast<hipStream_t>(stream)};
  gdsw::StreamMark mark_c{&M->coarse->stream_marks, static_cast<hipStream_t>(stream)};
  try {
    const gdsw::KrylovWs ws = gdsw::context_workspace(M->fine);
    const gdsw::Precond pc = [M](const double* v, double* z, hipStream_t s) { gdsw::mg_cycle(M, v, z, s); };
    return gdsw::solve_impl(M->fine, b, x, static_cast<hipStream_t>(stream), info, ws, false, &pc);
  } catch (const Error& e) {
    return gdsw::fail(e);
  }
}

int gdsw_mg_counts(gdsw_mg* M, int64_t* cycles, int64_t* coarse_iterations) {
  if (!M) {
    gdsw::g_last_error = "gdsw_mg_counts: NULL argument";
    return GDSW_EINVAL;
  }
  if (cycles) *cycles = M->cycles;
  if (coarse_iterations) *coarse_iterations = M->coarse_its;
  return GDSW_OK;
}

void gdsw_mg_destroy(gdsw_mg* M) {
  if (!M) return;
  delete M;                      // waits for the marks of its calls first (~gdsw_mg)
}

int gdsw_spmv(gdsw_ctx* C, const double* x, double* y, void* stream) {
  if (!C || !x || !y) {
    gdsw::g_last_error = "gdsw_spmv: NULL argument";
    return GDSW_EINVAL;
  }
  gdsw::StreamMark mark_{&C->stream_marks, static_cast<hipStream_t>(stream)};
  try {
    gdsw::spmv(C->levels[0].K, x, y, static_cast<hipStream_t>(stream));
  } catch (const Error& e) {
    return gdsw::fail(e);
  }
  return GDSW_OK;
}

int gdsw_scatter_local(gdsw_ctx* C, int32_t level, const double* w, double* z, void* stream) {
  if (!C || !w || !z || level < 1 || level > (int)C->levels.size()) {
    gdsw::g_last_error = "gdsw_scatter_local: bad argument";
    return GDSW_EINVAL;
  }
  gdsw::StreamMark mark_{&C->stream_marks, static_cast<hipStream_t>(stream)};
  try {
    gdsw::Level& L = C->levels[level - 1];
    gdsw::scatter_sum(L.n, L.sc_ptr, L.sc_pos, w, z, static_cast<hipStream_t>(stream));
  } catch (const Error& e) {
    return gdsw::fail(e);
  }
  return GDSW_OK;
}

static void fill_view(const gdsw::LevelMaps& m, int64_t n_dof, int nparts, gdsw_maps_view* out) {
  out->n_dof = (int32_t)n_dof;
  out->n_parts = nparts;
  out->dom_ptr = m.dom_ptr.data();
  out->dom = m.dom.data();
  out->int_ptr = m.int_ptr.data();
  out->inter = m.inter.data();
  out->n_gamma_nodes = (int32_t)m.gamma_nodes.size();
  out->gamma_nodes = m.gamma_nodes.data();
  out->n_entities = (int32_t)m.ent_kind.size();
  out->ent_ptr = m.ent_ptr.data();
  out->ent_nodes = m.ent_nodes.data();
  out->ent_kind = m.ent_kind.data();
  out->n_coarse = m.n_coarse;
  out->col_entity = m.col_entity.data();
  out->col_dir = m.col_dir.data();
  out->owner = m.owner.data();
}

int gdsw_export_maps(gdsw_ctx* C, int32_t level, gdsw_maps_view* out) {
  if (!C || !out || level < 1 || level > (int)C->levels.size()) {
    gdsw::g_last_error = "gdsw_export_maps: bad argument";
    return GDSW_EINVAL;
  }
  const gdsw::Level& L = C->levels[level - 1];
  fill_view(L.maps, L.n, L.nparts, out);
  return GDSW_OK;
}

struct gdsw_plan {
  gdsw::Plan P;
};

int gdsw_plan_create(const gdsw_problem* prob, const gdsw_options* opt, gdsw_plan** out) {
  if (!out) {
    gdsw::g_last_error = "out is NULL";
    return GDSW_EINVAL;
  }
  *out = nullptr;
  try {
    gdsw_options o;
    gdsw_default_options(&o);
    if (opt) o = *opt;
    gdsw_plan* p = new gdsw_plan();
    try {
      p->P = gdsw::plan_levels(prob, o);
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
  } catch (const Error& e) {
    return gdsw::fail(e);
  } catch (const std::bad_alloc&) {
    gdsw::g_last_error = "host allocation failed";
    return GDSW_ENOMEM;
  }
  return GDSW_OK;
}

int gdsw_plan_levels(gdsw_plan* plan, int32_t* schwarz_levels, int32_t* has_coarsest) {
  if (!plan) {
    gdsw::g_last_error = "plan is NULL";
    return GDSW_EINVAL;
  }
  if (schwarz_levels) *schwarz_levels = plan->P.schwarz;
  if (has_coarsest) *has_coarsest = plan->P.coarsest ? 1 : 0;
  return GDSW_OK;
}

int gdsw_plan_maps(gdsw_plan* plan, int32_t level, gdsw_maps_view* out) {
  if (!plan || !out || level < 1 || level > (int)plan->P.maps.size()) {
    gdsw::g_last_error = "gdsw_plan_maps: bad argument";
    return GDSW_EINVAL;
  }
  const gdsw::LevelMesh& mesh = plan->P.meshes[level - 1];
  fill_view(plan->P.maps[level - 1], mesh.n_dof, mesh.n_parts, out);
  return GDSW_OK;
}

void gdsw_plan_destroy(gdsw_plan* plan) { delete plan; }

int gdsw_get_stats(gdsw_ctx* C, gdsw_stats* out) {
  if (!C || !out) {
    gdsw::g_last_error = "gdsw_get_stats: NULL argument";
    return GDSW_EINVAL;
  }
  try {
    gdsw::drain_events(C);
  } catch (const Error& e) {
    return gdsw::fail(e);
  }
  *out = C->stats;
  return GDSW_OK;
}

size_t gdsw_footprint_bytes(const gdsw_problem* prob, const gdsw_options* opt) {
  try {
    gdsw_options o;
    gdsw_default_options(&o);
    if (opt) o = *opt;
    gdsw::Plan P = gdsw::plan_levels(prob, o);
    const size_t s = (o.precision == GDSW_MIXED) ? 4 : 8;
    size_t total = 0;
    size_t n_last = 0;
    for (size_t l = 0; l < P.maps.size(); ++l) {
      const gdsw::LevelMaps& m = P.maps[l];
      const size_t N = m.dom_ptr.size() - 1;
      size_t n2 = 0, sn = 0;
      for (size_t i = 0; i < N; ++i) {
        const size_t ni = (size_t)(m.dom_ptr[i + 1] - m.dom_ptr[i]);
        n2 += ni * (size_t)gdsw::lead_dim((int)ni, (int)(128 / s));
        sn += ni;
      }
      // factors, pivots / gather / local vectors, and the U12 scratch of the factorization
      total += n2 * s + sn * 24 + 128 * sn * s;
      size_t phi = 0;
      for (size_t i = 0; i < N; ++i)
        phi += (size_t)(m.int_ptr[i + 1] - m.int_ptr[i]) * (size_t)(m.pc_ptr[i + 1] - m.pc_ptr[i]);
      total += phi * (s + 8) + m.owner.size() * 24 + 128 * m.inter.size() * s;
      n_last = (size_t)m.n_coarse;
    }
    if (P.coarsest) total += 2 * n_last * n_last * 8 + 128 * n_last * 8;
    const size_t n = (size_t)prob->n;
    total += (size_t)(o.restart * 2 + 4) * n * 8;
    total += n / 3 + 512;                              // SpMV row-group flags
    return total;
  } catch (...) {
    return 0;
  }
}

void gdsw_destroy(gdsw_ctx* C) {
  if (!C) return;
  // the device blocks go back to the process cache: the context's destructor first waits for the
  // work of its calls (the mark recorded on every caller stream after each call, and its own
  // streams), so no queued work still uses them; other contexts' work is not waited for
  delete C;
}

}  // extern "C"
