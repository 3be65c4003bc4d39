// Host-side index maps of one GDSW level (section 2.1) and the coarse mesh
// that the recursion of section 2.2 works on.  Integer graph work only.
#include "maps.h"

#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <functional>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>

namespace gdsw {

namespace {

int host_threads() {
  if (const char* e = std::getenv("GDSW_HOST_THREADS")) {
    const int t = std::atoi(e);
    if (t >= 1) return t;
  }
  const unsigned hw = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(16u, hw));
}

// Process-wide worker threads for parallel_for (creating and joining threads
// per call costs a few hundred microseconds, and a setup makes dozens of calls).
// One caller at a time: run() returns false while another thread uses the pool.
// The pool is never destroyed (its threads live until the process ends); a
// forked child builds its own.
class HostPool {
 public:
  static HostPool* get(int workers) {
    static std::mutex mk;
    static HostPool* pool = nullptr;
    static pid_t owner = 0;
    std::lock_guard<std::mutex> lk(mk);
    if (!pool || owner != getpid()) {
      pool = new HostPool(workers);
      owner = getpid();
    }
    return pool;
  }
  // work(t) for t in [0, nthreads) (the caller runs t = 0); false if busy
  bool run(int nthreads, const std::function<void(int)>& work) {
    std::unique_lock<std::mutex> busy(busy_, std::try_to_lock);
    if (!busy.owns_lock()) return false;
    const int want = std::min(nthreads, (int)workers_.size() + 1);
    {
      std::lock_guard<std::mutex> lk(m_);
      job_ = &work;
      want_ = want;
      pending_ = want - 1;
      ++gen_;
    }
    cv_.notify_all();
    work(0);
    std::unique_lock<std::mutex> lk(m_);
    done_.wait(lk, [&] { return pending_ == 0; });
    job_ = nullptr;
    return true;
  }

 private:
  explicit HostPool(int workers) {
    for (int t = 1; t <= workers; ++t) workers_.emplace_back([this, t] { loop(t); });
  }
  void loop(int id) {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> lk(m_);
    for (;;) {
      cv_.wait(lk, [&] { return gen_ != seen; });
      seen = gen_;
      if (id >= want_) continue;
      const std::function<void(int)>* job = job_;
      lk.unlock();
      (*job)(id);
      lk.lock();
      if (--pending_ == 0) done_.notify_one();
    }
  }
  std::mutex busy_, m_;
  std::condition_variable cv_, done_;
  std::vector<std::thread> workers_;
  const std::function<void(int)>* job_ = nullptr;
  uint64_t gen_ = 0;
  int want_ = 0, pending_ = 0;
};

// f(thread, begin, end) over [0, n) in dynamically scheduled chunks.
template <typename F>
void parallel_for(int n, int nthreads, F f) {
  if (n <= 0) return;
  if (nthreads <= 1 || n < 64) {
    f(0, 0, n);
    return;
  }
  std::atomic<int> next(0);
  const int chunk = std::max(8, n / (nthreads * 8));
  const std::function<void(int)> work = [&](int t) {
    for (;;) {
      const int b = next.fetch_add(chunk);
      if (b >= n) break;
      f(t, b, std::min(n, b + chunk));
    }
  };
  if (HostPool::get(host_threads() - 1)->run(nthreads, work)) return;
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& th : pool) th.join();
}

// Sort and deduplicate each segment of a CSR list (segments in parallel), then
// compact in place.
template <typename V>
void sort_unique_segments(std::vector<int64_t>& ptr, V& val) {
  const int nseg = (int)ptr.size() - 1;
  if (nseg <= 0) return;
  std::vector<int> cnt(nseg);
  parallel_for(nseg, host_threads(), [&](int, int s0, int s1) {
    for (int s = s0; s < s1; ++s) {
      auto a = val.begin() + ptr[s], b = val.begin() + ptr[s + 1];
      std::sort(a, b);
      cnt[s] = (int)(std::unique(a, b) - a);
    }
  });
  int64_t w = 0;
  for (int s = 0; s < nseg; ++s) {          // forward: the write position never passes the read one
    const int64_t a = ptr[s];
    ptr[s] = w;
    for (int k = 0; k < cnt[s]; ++k) val[w++] = val[a + k];
  }
  ptr[nseg] = w;
  val.resize(w);
}

// v = n copies of x, written in parallel
void fill_n_parallel(RawVec<int>& v, int64_t n, int x) {
  v.resize(n);
  parallel_for((int)((n + 4095) / 4096), host_threads(), [&](int, int b0, int b1) {
    std::fill(v.begin() + (int64_t)b0 * 4096, v.begin() + std::min<int64_t>(n, (int64_t)b1 * 4096), x);
  });
}

// True when the non-negative entries of ids, in array order, are strictly increasing.
bool increasing_free(const std::vector<int>& ids) {
  const int n = (int)ids.size();
  const int nchunk = (n + 65535) / 65536;
  if (nchunk == 0) return true;
  std::vector<int> first(nchunk, -1), last(nchunk, -1);
  std::atomic<bool> ok(true);
  parallel_for(nchunk, host_threads(), [&](int, int c0, int c1) {
    for (int c = c0; c < c1; ++c) {
      int prev = -1;
      for (int k = c * 65536; k < std::min(n, (c + 1) * 65536); ++k) {
        const int g = ids[k];
        if (g < 0) continue;
        if (prev >= 0 && g <= prev) ok = false;
        if (first[c] < 0) first[c] = g;
        prev = g;
      }
      last[c] = prev;
    }
  });
  int prev = -1;
  for (int c = 0; c < nchunk; ++c) {
    if (first[c] < 0) continue;
    if (prev >= 0 && first[c] <= prev) return false;
    prev = last[c];
  }
  return ok.load();
}

// elements containing each node (CSR, ascending), for meshes whose builder did not make them
void node_elements(const LevelMesh& mesh, std::vector<int64_t>& ptr, RawVec<int>& el) {
  ptr.assign(mesh.n_nodes + 1, 0);
  for (int e = 0; e < mesh.n_elem; ++e)
    for (int64_t k = mesh.en_ptr[e]; k < mesh.en_ptr[e + 1]; ++k) ptr[mesh.en[k] + 1]++;
  for (int v = 0; v < mesh.n_nodes; ++v) ptr[v + 1] += ptr[v];
  el.assign(ptr[mesh.n_nodes], 0);
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (int e = 0; e < mesh.n_elem; ++e)
    for (int64_t k = mesh.en_ptr[e]; k < mesh.en_ptr[e + 1]; ++k) el[fill[mesh.en[k]]++] = e;
}

bool same_set(const LevelMaps& m, int u, int v) {
  const int64_t a0 = m.s_ptr[u], a1 = m.s_ptr[u + 1], b0 = m.s_ptr[v], b1 = m.s_ptr[v + 1];
  if (a1 - a0 != b1 - b0) return false;
  for (int64_t k = 0; k < a1 - a0; ++k)
    if (m.s[a0 + k] != m.s[b0 + k]) return false;
  return true;
}

}  // namespace

void host_parallel(int nthreads, const std::function<void(int)>& work) {
  nthreads = std::max(1, std::min(nthreads, host_threads()));
  if (nthreads == 1) {
    work(0);
    return;
  }
  if (HostPool::get(host_threads() - 1)->run(nthreads, work)) return;
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& th : pool) th.join();
}

int host_thread_count() { return host_threads(); }

std::string build_level1_mesh(int64_t n, int n_nodes, const int* node_dof, int n_elem,
                              const int* elem_node, const int* elem_pdof, const int* elem_part,
                              int n_parts, LevelMesh& out) {
  if (n <= 0 || n > INT32_MAX) return "n out of range";
  if (n_nodes <= 0 || n_elem <= 0 || n_parts <= 0) return "empty mesh or partition";
  out.n_dof = (int)n;
  out.n_nodes = n_nodes;
  out.node_dof.assign(node_dof, node_dof + (size_t)n_nodes * 3);
  out.n_elem = n_elem;
  const int nt = host_threads();
  out.en.resize((size_t)n_elem * 27);
  parallel_for(n_elem, nt, [&](int, int e0, int e1) {
    std::copy(elem_node + (size_t)e0 * 27, elem_node + (size_t)e1 * 27, out.en.begin() + (size_t)e0 * 27);
  });
  out.en_ptr.resize(n_elem + 1);
  for (int e = 0; e <= n_elem; ++e) out.en_ptr[e] = (int64_t)e * 27;
  out.elem_pdof.assign(elem_pdof, elem_pdof + (size_t)n_elem * 4);
  out.elem_part.assign(elem_part, elem_part + n_elem);
  out.n_parts = n_parts;
  // every free dof exactly once: node_dof marked first, then elem_pdof (in parallel; the second mark
  // of an id, whichever thread makes it, is a repeat)
  std::unique_ptr<std::atomic<unsigned char>[]> seen(new std::atomic<unsigned char>[n]);
  parallel_for((int)n, nt, [&](int, int g0, int g1) {
    for (int g = g0; g < g1; ++g) seen[g].store(0, std::memory_order_relaxed);
  });
  std::atomic<bool> bad(false);
  auto mark_all = [&](const std::vector<int>& ids) {
    parallel_for((int)ids.size(), nt, [&](int, int k0, int k1) {
      for (int k = k0; k < k1; ++k) {
        const int g = ids[k];
        if (g < -1 || g >= n || (g >= 0 && seen[g].exchange(1, std::memory_order_relaxed))) bad = true;
      }
    });
    return !bad.load();
  };
  if (!mark_all(out.node_dof)) return "node_dof: id out of range or repeated";
  if (!mark_all(out.elem_pdof)) return "elem_pdof: id out of range or repeated";
  std::atomic<int64_t> missing(n);
  parallel_for((int)n, nt, [&](int, int g0, int g1) {
    for (int g = g0; g < g1; ++g)
      if (!seen[g].load(std::memory_order_relaxed)) {
        int64_t cur = missing.load();
        while (g < cur && !missing.compare_exchange_weak(cur, g)) {
        }
      }
  });
  if (missing.load() < n) return "dof " + std::to_string(missing.load()) + " is not referenced by node_dof/elem_pdof";
  parallel_for(n_elem, nt, [&](int, int e0, int e1) {
    for (size_t k = (size_t)e0 * 27; k < (size_t)e1 * 27; ++k)
      if (out.en[k] < 0 || out.en[k] >= n_nodes) bad = true;
  });
  if (bad.load()) return "elem_node: node id out of range";
  std::vector<int> cnt(n_parts, 0);
  for (int p : out.elem_part) {
    if (p < 0 || p >= n_parts) return "elem_part: part id out of range";
    cnt[p]++;
  }
  for (int i = 0; i < n_parts; ++i)
    if (!cnt[i]) return "level-1 part " + std::to_string(i) + " has no element";
  // node graph: two nodes of one element whose lattice offsets differ by at most one per axis
  // (at most 26 neighbours per node), built node by node from the elements holding it
  // node -> (element, position) lists, ascending by element then position: counted and filled in
  // parallel with per-node atomic counters, then each node's few entries sorted
  std::vector<int64_t> ne_ptr(n_nodes + 1, 0);
  RawVec<int> ne_el, ne_loc;
  {
    std::unique_ptr<std::atomic<int>[]> c(new std::atomic<int>[n_nodes]);
    auto zero = [&] {
      parallel_for(n_nodes, nt, [&](int, int v0, int v1) {
        for (int v = v0; v < v1; ++v) c[v].store(0, std::memory_order_relaxed);
      });
    };
    zero();
    parallel_for(n_elem, nt, [&](int, int e0, int e1) {
      for (size_t k = (size_t)e0 * 27; k < (size_t)e1 * 27; ++k) c[out.en[k]].fetch_add(1, std::memory_order_relaxed);
    });
    for (int v = 0; v < n_nodes; ++v) ne_ptr[v + 1] = ne_ptr[v] + c[v].load(std::memory_order_relaxed);
    ne_el.resize(ne_ptr[n_nodes]);
    ne_loc.resize(ne_ptr[n_nodes]);
    zero();
    parallel_for(n_elem, nt, [&](int, int e0, int e1) {
      for (int e = e0; e < e1; ++e)
        for (int a = 0; a < 27; ++a) {
          const int v = out.en[(size_t)e * 27 + a];
          const int64_t q = ne_ptr[v] + c[v].fetch_add(1, std::memory_order_relaxed);
          ne_el[q] = e;
          ne_loc[q] = a;
        }
    });
    parallel_for(n_nodes, nt, [&](int, int v0, int v1) {
      for (int v = v0; v < v1; ++v)
        for (int64_t q = ne_ptr[v] + 1; q < ne_ptr[v + 1]; ++q) {   // insertion sort by (element, position)
          const int e = ne_el[q], a = ne_loc[q];
          int64_t r = q;
          while (r > ne_ptr[v] && (ne_el[r - 1] > e || (ne_el[r - 1] == e && ne_loc[r - 1] > a))) {
            ne_el[r] = ne_el[r - 1];
            ne_loc[r] = ne_loc[r - 1];
            --r;
          }
          ne_el[r] = e;
          ne_loc[r] = a;
        }
    });
  }
  constexpr int MAXNB = 26;
  // the positions of a 27-node element within one lattice step of each position, ascending
  struct Near {
    int count;
    int pos[26];
  };
  static const std::vector<Near> near = [] {
    std::vector<Near> t(27);
    for (int a = 0; a < 27; ++a) {
      t[a].count = 0;
      for (int b = 0; b < 27; ++b) {
        if (b == a) continue;
        const int dx = a % 3 - b % 3, dy = (a / 3) % 3 - (b / 3) % 3, dz = a / 9 - b / 9;
        if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) t[a].pos[t[a].count++] = b;
      }
    }
    return t;
  }();
  std::unique_ptr<int[]> nbuf(new int[(size_t)n_nodes * MAXNB]);   // every row written before it is read
  std::vector<int> ncount(n_nodes, 0);
  std::atomic<bool> overflow(false);
  // distinct candidates through a per-thread stamp (stamp[w] == v: w already taken for node v), then
  // the at most 26 neighbours sorted
  std::vector<std::vector<int>> nstamp(nt);
  parallel_for(n_nodes, nt, [&](int th, int v0, int v1) {
    std::vector<int>& stamp = nstamp[th];
    if (stamp.empty()) stamp.assign(n_nodes, -1);
    for (int v = v0; v < v1; ++v) {
      if (ne_ptr[v + 1] - ne_ptr[v] > 8) {      // a hexahedral lattice node lies in at most 8 elements
        overflow = true;
        continue;
      }
      int* row = nbuf.get() + (size_t)v * MAXNB;
      int w = 0;
      for (int64_t q = ne_ptr[v]; q < ne_ptr[v + 1] && w <= MAXNB; ++q) {
        const int* el = out.en.data() + (size_t)ne_el[q] * 27;
        const Near& t = near[ne_loc[q]];
        for (int k = 0; k < t.count; ++k) {
          const int c = el[t.pos[k]];
          if (stamp[c] == v) continue;
          stamp[c] = v;
          if (w == MAXNB) {
            overflow = true;
            w = MAXNB + 1;
            break;
          }
          row[w++] = c;
        }
      }
      if (w > MAXNB) continue;
      std::sort(row, row + w);
      ncount[v] = w;
    }
  });
  if (overflow) return "elem_node: a node lies in more than 8 elements or has more than 26 lattice neighbours";
  std::vector<int64_t> cntp(n_nodes + 1, 0);
  for (int v = 0; v < n_nodes; ++v) cntp[v + 1] = cntp[v] + ncount[v];
  RawVec<int> nb(cntp[n_nodes]);
  parallel_for(n_nodes, host_threads(), [&](int, int v0, int v1) {
    for (int v = v0; v < v1; ++v)
      std::copy(nbuf.get() + (size_t)v * MAXNB, nbuf.get() + (size_t)v * MAXNB + ncount[v], nb.begin() + cntp[v]);
  });
  out.adj_ptr = std::move(cntp);
  out.adj = std::move(nb);
  out.ne_ptr = std::move(ne_ptr);
  out.ne = std::move(ne_el);
  return "";
}

void build_domains(const LevelMesh& mesh, int delta, LevelMaps& m) {
  const int N = mesh.n_parts;
  const int nn = mesh.n_nodes;
  std::vector<int64_t> ne_ptr_own;
  RawVec<int> ne_own;
  if (mesh.ne_ptr.empty()) node_elements(mesh, ne_ptr_own, ne_own);
  const std::vector<int64_t>& ne_ptr = mesh.ne_ptr.empty() ? ne_ptr_own : mesh.ne_ptr;
  const RawVec<int>& ne = mesh.ne_ptr.empty() ? ne_own : mesh.ne;
  // S(v)
  m.s_ptr = ne_ptr;
  m.s.resize(ne.size());
  parallel_for(nn, host_threads(), [&](int, int v0, int v1) {
    for (int64_t k = ne_ptr[v0]; k < ne_ptr[v1]; ++k) m.s[k] = mesh.elem_part[ne[k]];
  });
  sort_unique_segments(m.s_ptr, m.s);
  // owning part of every dof (restricted combination): first part of S(v), the element's part for pressure
  fill_n_parallel(m.owner, mesh.n_dof, -1);
  parallel_for(nn, host_threads(), [&](int, int v0, int v1) {     // every dof has one node or element
    for (int v = v0; v < v1; ++v) {
      if (m.s_ptr[v + 1] == m.s_ptr[v]) continue;
      const int own = m.s[m.s_ptr[v]];
      for (int d = 0; d < 3; ++d) {
        const int g = mesh.node_dof[3 * v + d];
        if (g >= 0) m.owner[g] = own;
      }
    }
  });
  parallel_for(mesh.n_elem, host_threads(), [&](int, int e0, int e1) {
    for (int e = e0; e < e1; ++e)
      for (int q = 0; q < 4; ++q) {
        const int g = mesh.elem_pdof[4 * e + q];
        if (g >= 0) m.owner[g] = mesh.elem_part[e];
      }
  });
  // D_i: nodes of the part's elements grown by delta node-graph layers, plus its pressure dofs
  std::vector<std::vector<int>> part_elems(N);
  for (int e = 0; e < mesh.n_elem; ++e) part_elems[mesh.elem_part[e]].push_back(e);
  std::vector<std::vector<int>> dofs(N);
  const int nthreads = host_threads();
  // When the velocity dofs grow with (node, component) and the pressure dofs with (element, mode),
  // a part's sorted dof list is the merge of its velocity dofs in node order and its pressure dofs
  // in element order: sorting the nodes (a third as many) replaces sorting the dofs.
  const bool by_node = increasing_free(mesh.node_dof), by_elem = increasing_free(mesh.elem_pdof);
  std::vector<std::vector<int>> stamps(nthreads);
  parallel_for(N, nthreads, [&](int t, int i0, int i1) {
    std::vector<int>& stamp = stamps[t];
    if (stamp.empty()) stamp.assign(nn, -1);
    std::vector<int> layer, frontier, next, vel, prs;
    for (int i = i0; i < i1; ++i) {
      std::vector<int>& o = dofs[i];
      layer.clear();
      for (int e : part_elems[i])
        for (int64_t k = mesh.en_ptr[e]; k < mesh.en_ptr[e + 1]; ++k) {
          const int v = mesh.en[k];
          if (stamp[v] != i) {
            stamp[v] = i;
            layer.push_back(v);
          }
        }
      frontier.assign(layer.begin(), layer.end());
      for (int l = 0; l < delta; ++l) {
        next.clear();
        for (int u : frontier)
          for (int64_t k = mesh.adj_ptr[u]; k < mesh.adj_ptr[u + 1]; ++k) {
            const int w = mesh.adj[k];
            if (stamp[w] != i) {
              stamp[w] = i;
              next.push_back(w);
            }
          }
        layer.insert(layer.end(), next.begin(), next.end());
        frontier.swap(next);
      }
      if (by_node && by_elem) {
        std::sort(layer.begin(), layer.end());
        vel.clear();
        prs.clear();
        for (int v : layer)
          for (int d = 0; d < 3; ++d) {
            const int g = mesh.node_dof[3 * v + d];
            if (g >= 0) vel.push_back(g);
          }
        for (int e : part_elems[i])              // elements ascending
          for (int q = 0; q < 4; ++q) {
            const int g = mesh.elem_pdof[4 * e + q];
            if (g >= 0) prs.push_back(g);
          }
        o.resize(vel.size() + prs.size());
        std::merge(vel.begin(), vel.end(), prs.begin(), prs.end(), o.begin());
        continue;
      }
      for (int v : layer)
        for (int d = 0; d < 3; ++d) {
          const int g = mesh.node_dof[3 * v + d];
          if (g >= 0) o.push_back(g);
        }
      for (int e : part_elems[i])
        for (int q = 0; q < 4; ++q) {
          const int g = mesh.elem_pdof[4 * e + q];
          if (g >= 0) o.push_back(g);
        }
      std::sort(o.begin(), o.end());
    }
  });
  m.dom_ptr.assign(N + 1, 0);
  for (int i = 0; i < N; ++i) m.dom_ptr[i + 1] = m.dom_ptr[i] + (int64_t)dofs[i].size();
  m.dom.resize(m.dom_ptr[N]);
  parallel_for(N, nthreads, [&](int, int i0, int i1) {
    for (int i = i0; i < i1; ++i) std::copy(dofs[i].begin(), dofs[i].end(), m.dom.begin() + m.dom_ptr[i]);
  });
}

void build_maps(const LevelMesh& mesh, int delta, LevelMaps& m, bool linear_interior) {
  const int N = mesh.n_parts;
  const int nn = mesh.n_nodes;
  if ((int)m.dom_ptr.size() != N + 1) build_domains(mesh, delta, m);
  auto nS = [&](int v) { return m.s_ptr[v + 1] - m.s_ptr[v]; };
  auto has_free = [&](int v) {
    return mesh.node_dof[3 * v] >= 0 || mesh.node_dof[3 * v + 1] >= 0 || mesh.node_dof[3 * v + 2] >= 0;
  };
  // interface nodes and entities (components of equal-S classes, in order of their smallest node)
  m.gamma_nodes.clear();
  for (int v = 0; v < nn; ++v)
    if (has_free(v) && nS(v) >= 2) m.gamma_nodes.push_back(v);
  m.node_ent.assign(nn, -1);
  std::vector<char> is_gamma(nn, 0);
  for (int v : m.gamma_nodes) is_gamma[v] = 1;
  // entities: connected components of the interface nodes under "adjacent with the same S",
  // numbered in order of their smallest node.  Parallel union-find that links the larger root
  // below the smaller one, so every component's root is its smallest node.
  const int ng = (int)m.gamma_nodes.size();
  const int nth = host_threads();
  std::unique_ptr<std::atomic<int>[]> parent(new std::atomic<int>[nn]);
  parallel_for(ng, nth, [&](int, int k0, int k1) {
    for (int k = k0; k < k1; ++k) parent[m.gamma_nodes[k]].store(m.gamma_nodes[k], std::memory_order_relaxed);
  });
  auto find = [&](int x) {
    for (;;) {
      int p = parent[x].load(std::memory_order_relaxed);
      if (p == x) return x;
      const int gp = parent[p].load(std::memory_order_relaxed);
      if (gp != p) parent[x].compare_exchange_weak(p, gp, std::memory_order_relaxed);   // path halving
      x = p;
    }
  };
  parallel_for(ng, nth, [&](int, int k0, int k1) {
    for (int k = k0; k < k1; ++k) {
      const int u = m.gamma_nodes[k];
      for (int64_t q = mesh.adj_ptr[u]; q < mesh.adj_ptr[u + 1]; ++q) {
        const int w = mesh.adj[q];
        if (w <= u || !is_gamma[w] || !same_set(m, u, w)) continue;
        for (;;) {
          int a = find(u), b = find(w);
          if (a == b) break;
          if (a > b) std::swap(a, b);
          if (parent[b].compare_exchange_strong(b, a, std::memory_order_relaxed)) break;   // b stays a root until linked
        }
      }
    }
  });
  std::vector<int> root(ng);
  parallel_for(ng, nth, [&](int, int k0, int k1) {
    for (int k = k0; k < k1; ++k) root[k] = find(m.gamma_nodes[k]);
  });
  m.ent_kind.clear();
  std::vector<int64_t> ecount;
  for (int k = 0; k < ng; ++k) {                      // gamma nodes ascending: roots open entities in order
    const int u = m.gamma_nodes[k];
    if (root[k] == u) {
      m.node_ent[u] = (int)ecount.size();
      ecount.push_back(0);
    }
  }
  for (int k = 0; k < ng; ++k) {
    const int E = m.node_ent[root[k]];
    m.node_ent[m.gamma_nodes[k]] = E;
    ecount[E]++;
  }
  const int ne_ = (int)ecount.size();
  m.ent_ptr.assign(ne_ + 1, 0);
  for (int E = 0; E < ne_; ++E) m.ent_ptr[E + 1] = m.ent_ptr[E] + ecount[E];
  m.ent_nodes.resize(m.ent_ptr[ne_]);
  {
    std::vector<int64_t> fill(m.ent_ptr.begin(), m.ent_ptr.end() - 1);
    for (int u : m.gamma_nodes) m.ent_nodes[fill[m.node_ent[u]]++] = u;   // ascending within each entity
  }
  m.ent_kind.resize(ne_);
  for (int E = 0; E < ne_; ++E) {
    const int v = m.ent_nodes[m.ent_ptr[E]];
    m.ent_kind[E] = ecount[E] == 1 ? 0 : (nS(v) == 2 ? 2 : 1);
  }
  const int n_ent = (int)m.ent_kind.size();
  m.es_ptr.assign(n_ent + 1, 0);
  m.es.clear();
  for (int E = 0; E < n_ent; ++E) {
    const int v = m.ent_nodes[m.ent_ptr[E]];
    for (int64_t k = m.s_ptr[v]; k < m.s_ptr[v + 1]; ++k) m.es.push_back(m.s[k]);
    m.es_ptr[E + 1] = (int64_t)m.es.size();
  }
  // coarse columns: (entity, direction) with a free dof, then one pressure column per part
  // (counted in parallel, numbered in (entity, direction) order, then filled and sorted in parallel)
  std::vector<int> ecnt((size_t)n_ent * 3);
  parallel_for(n_ent, host_threads(), [&](int, int E0, int E1) {
    for (int E = E0; E < E1; ++E)
      for (int d = 0; d < 3; ++d) {
        int c = 0;
        for (int64_t k = m.ent_ptr[E]; k < m.ent_ptr[E + 1]; ++k) c += mesh.node_dof[3 * m.ent_nodes[k] + d] >= 0;
        ecnt[(size_t)E * 3 + d] = c;
      }
  });
  m.col_entity.clear();
  m.col_dir.clear();
  m.col_ptr.assign(1, 0);
  m.ent_col.assign((size_t)n_ent * 3, -1);
  for (int E = 0; E < n_ent; ++E)
    for (int d = 0; d < 3; ++d) {
      const int c = ecnt[(size_t)E * 3 + d];
      if (!c) continue;
      m.ent_col[(size_t)E * 3 + d] = (int)m.col_entity.size();
      m.col_entity.push_back(E);
      m.col_dir.push_back(d);
      m.col_ptr.push_back(m.col_ptr.back() + c);
    }
  m.col_dofs.resize(m.col_ptr.back());
  parallel_for(n_ent, host_threads(), [&](int, int E0, int E1) {
    for (int E = E0; E < E1; ++E)
      for (int d = 0; d < 3; ++d) {
        const int col = m.ent_col[(size_t)E * 3 + d];
        if (col < 0) continue;
        int64_t w = m.col_ptr[col];
        for (int64_t k = m.ent_ptr[E]; k < m.ent_ptr[E + 1]; ++k) {
          const int g = mesh.node_dof[3 * m.ent_nodes[k] + d];
          if (g >= 0) m.col_dofs[w++] = g;
        }
        std::sort(m.col_dofs.begin() + m.col_ptr[col], m.col_dofs.begin() + w);
      }
  });
  std::vector<std::vector<int>> part_elems(N);
  for (int e = 0; e < mesh.n_elem; ++e) part_elems[mesh.elem_part[e]].push_back(e);
  m.part_col.assign(N, -1);
  for (int i = 0; i < N; ++i) {
    const size_t before = m.col_dofs.size();
    for (int e : part_elems[i]) {
      const int g = mesh.elem_pdof[4 * e];
      if (g >= 0) m.col_dofs.push_back(g);
    }
    if (m.col_dofs.size() > before) {
      std::sort(m.col_dofs.begin() + before, m.col_dofs.end());
      m.part_col[i] = (int)m.col_entity.size();
      m.col_entity.push_back(-1 - i);
      m.col_dir.push_back(3);
      m.col_ptr.push_back((int64_t)m.col_dofs.size());
    }
  }
  m.n_coarse = (int)m.col_entity.size();
  // per-dof tables
  const int n = mesh.n_dof;
  fill_n_parallel(m.dof_gcol, n, -1);
  fill_n_parallel(m.dof_ipart, n, -1);
  fill_n_parallel(m.dof_irow, n, -1);
  parallel_for((int)m.gamma_nodes.size(), host_threads(), [&](int, int k0, int k1) {   // distinct dofs
    for (int k = k0; k < k1; ++k) {
      const int v = m.gamma_nodes[k];
      for (int d = 0; d < 3; ++d) {
        const int g = mesh.node_dof[3 * v + d];
        if (g >= 0) m.dof_gcol[g] = m.ent_col[(size_t)m.node_ent[v] * 3 + d];
      }
    }
  });
  parallel_for(mesh.n_elem, host_threads(), [&](int, int e0, int e1) {
    for (int e = e0; e < e1; ++e) {
      const int g = mesh.elem_pdof[4 * e];
      if (g >= 0) m.dof_gcol[g] = m.part_col[mesh.elem_part[e]];
    }
  });
  // interior sets and coarse columns, part by part (in parallel; concatenated in part order)
  struct PartOut {
    std::vector<int> idofs, pcols, z_lc, z_dof;
  };
  std::vector<PartOut> outp(N);
  const int nthreads = host_threads();
  // With dof ids growing with (node, component) and (element, mode), the sorted lists below come from
  // the closure's nodes in sorted order and the part's elements in order (merges and a counting sort
  // by local column) instead of sorts of the dof lists; other numberings take the sorting path.
  const bool by_order = increasing_free(mesh.node_dof) && increasing_free(mesh.elem_pdof);
  std::vector<std::vector<int>> stamps(nthreads), cstamps(nthreads), cposs(nthreads);
  parallel_for(N, nthreads, [&](int t, int i0, int i1) {
    std::vector<int>& stamp = stamps[t];
    if (stamp.empty()) stamp.assign(nn, -1);
    std::vector<int> layer, ivel, iprs, zv, zp, zall, ccnt;
    std::vector<std::pair<int, int>> zs;
    for (int i = i0; i < i1; ++i) {
      PartOut& o = outp[i];
      layer.clear();
      for (int e : part_elems[i])
        for (int64_t k = mesh.en_ptr[e]; k < mesh.en_ptr[e + 1]; ++k) {
          const int v = mesh.en[k];
          if (stamp[v] != i) {
            stamp[v] = i;
            layer.push_back(v);
          }
        }
      if (by_order) {
        std::vector<int>& cstamp = cstamps[t];
        std::vector<int>& cpos = cposs[t];
        if (cstamp.empty()) {
          cstamp.assign(m.n_coarse, -1);
          cpos.assign(m.n_coarse, 0);
        }
        std::sort(layer.begin(), layer.end());
        ivel.clear();
        iprs.clear();
        zv.clear();
        zp.clear();
        for (int v : layer) {
          const bool interior = nS(v) == 1 && m.s[m.s_ptr[v]] == i;
          for (int d = 0; d < 3; ++d) {
            const int g = mesh.node_dof[3 * v + d];
            if (g < 0) continue;
            if (interior) ivel.push_back(g);
            else if (is_gamma[v]) zv.push_back(g);
          }
        }
        for (int e : part_elems[i])              // elements ascending
          for (int q = 0; q < 4; ++q) {
            const int g = mesh.elem_pdof[4 * e + q];
            if (g < 0) continue;
            if (q > 0) {
              if (linear_interior) iprs.push_back(g);
            } else {
              zp.push_back(g);
            }
          }
        o.idofs.resize(ivel.size() + iprs.size());
        std::merge(ivel.begin(), ivel.end(), iprs.begin(), iprs.end(), o.idofs.begin());
        for (size_t a = 0; a < o.idofs.size(); ++a) {   // interior dofs belong to one part only
          m.dof_ipart[o.idofs[a]] = i;
          m.dof_irow[o.idofs[a]] = (int)a;
        }
        zall.resize(zv.size() + zp.size());
        std::merge(zv.begin(), zv.end(), zp.begin(), zp.end(), zall.begin());
        for (int g : zall) {                      // coarse columns of the part, sorted
          const int c = m.dof_gcol[g];
          if (cstamp[c] != i) {
            cstamp[c] = i;
            o.pcols.push_back(c);
          }
        }
        std::sort(o.pcols.begin(), o.pcols.end());
        const int mi = (int)o.pcols.size();
        for (int a = 0; a < mi; ++a) cpos[o.pcols[a]] = a;
        ccnt.assign(mi + 1, 0);                   // interface dofs by (local column, dof): a stable
        for (int g : zall) ccnt[cpos[m.dof_gcol[g]] + 1]++;   // counting sort of the ascending dofs
        for (int a = 0; a < mi; ++a) ccnt[a + 1] += ccnt[a];
        o.z_lc.resize(zall.size());
        o.z_dof.resize(zall.size());
        for (int g : zall) {
          const int lc = cpos[m.dof_gcol[g]];
          const int at = ccnt[lc]++;
          o.z_lc[at] = lc;
          o.z_dof[at] = g;
        }
        continue;
      }
      const size_t n_closure = layer.size();
      zs.clear();
      for (size_t k = 0; k < n_closure; ++k) {
        const int v = layer[k];
        const bool interior = nS(v) == 1 && m.s[m.s_ptr[v]] == i;
        for (int d = 0; d < 3; ++d) {
          const int g = mesh.node_dof[3 * v + d];
          if (g < 0) continue;
          if (interior) o.idofs.push_back(g);
          else if (is_gamma[v]) zs.push_back({m.dof_gcol[g], g});
        }
      }
      for (int e : part_elems[i])
        for (int q = 0; q < 4; ++q) {
          const int g = mesh.elem_pdof[4 * e + q];
          if (g < 0) continue;
          if (q > 0) {
            if (linear_interior) o.idofs.push_back(g);
          } else {
            zs.push_back({m.dof_gcol[g], g});
          }
        }
      std::sort(o.idofs.begin(), o.idofs.end());
      for (size_t a = 0; a < o.idofs.size(); ++a) {   // interior dofs belong to one part only
        m.dof_ipart[o.idofs[a]] = i;
        m.dof_irow[o.idofs[a]] = (int)a;
      }
      // coarse columns of the part: every column of an interface dof in its closure
      for (auto& z : zs) o.pcols.push_back(z.first);
      std::sort(o.pcols.begin(), o.pcols.end());
      o.pcols.erase(std::unique(o.pcols.begin(), o.pcols.end()), o.pcols.end());
      // interface dofs of the closure, keyed by their local column
      for (auto& z : zs) z.first = (int)(std::lower_bound(o.pcols.begin(), o.pcols.end(), z.first) - o.pcols.begin());
      std::sort(zs.begin(), zs.end());
      for (auto& z : zs) {
        o.z_lc.push_back(z.first);
        o.z_dof.push_back(z.second);
      }
    }
  });
  m.int_ptr.assign(N + 1, 0);
  m.pc_ptr.assign(N + 1, 0);
  m.z_ptr.assign(N + 1, 0);
  for (int i = 0; i < N; ++i) {
    m.int_ptr[i + 1] = m.int_ptr[i] + (int64_t)outp[i].idofs.size();
    m.pc_ptr[i + 1] = m.pc_ptr[i] + (int64_t)outp[i].pcols.size();
    m.z_ptr[i + 1] = m.z_ptr[i] + (int64_t)outp[i].z_dof.size();
  }
  m.inter.resize(m.int_ptr[N]);
  m.pcols.resize(m.pc_ptr[N]);
  m.z_dof.resize(m.z_ptr[N]);
  m.z_lc.resize(m.z_ptr[N]);
  parallel_for(N, nthreads, [&](int, int i0, int i1) {
    for (int i = i0; i < i1; ++i) {
      const PartOut& o = outp[i];
      std::copy(o.idofs.begin(), o.idofs.end(), m.inter.begin() + m.int_ptr[i]);
      std::copy(o.pcols.begin(), o.pcols.end(), m.pcols.begin() + m.pc_ptr[i]);
      std::copy(o.z_dof.begin(), o.z_dof.end(), m.z_dof.begin() + m.z_ptr[i]);
      std::copy(o.z_lc.begin(), o.z_lc.end(), m.z_lc.begin() + m.z_ptr[i]);
    }
  });
  // per coarse column: the parts that hold it
  std::vector<int64_t> cnt(m.n_coarse + 1, 0);
  for (int i = 0; i < N; ++i)
    for (int64_t k = m.pc_ptr[i]; k < m.pc_ptr[i + 1]; ++k) cnt[m.pcols[k] + 1]++;
  for (int c = 0; c < m.n_coarse; ++c) cnt[c + 1] += cnt[c];
  m.cp_ptr = cnt;
  m.cp_part.assign(cnt[m.n_coarse], 0);
  m.cp_lc.assign(cnt[m.n_coarse], 0);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int i = 0; i < N; ++i)
    for (int64_t k = m.pc_ptr[i]; k < m.pc_ptr[i + 1]; ++k) {
      const int c = m.pcols[k];
      m.cp_part[fill[c]] = i;
      m.cp_lc[fill[c]] = (int)(k - m.pc_ptr[i]);
      fill[c]++;
    }
}

std::string build_next_mesh(const LevelMesh& mesh, const LevelMaps& m, const int* parent,
                            int n_parts_next, LevelMesh& out) {
  const int n_ent = (int)m.ent_kind.size();
  const int N = mesh.n_parts;
  out.n_dof = m.n_coarse;
  out.n_nodes = n_ent;
  out.node_dof = m.ent_col;
  out.n_elem = N;
  // element i's nodes: entities E with i in S(E), ascending
  std::vector<int64_t> cnt(N + 1, 0);
  for (int E = 0; E < n_ent; ++E)
    for (int64_t k = m.es_ptr[E]; k < m.es_ptr[E + 1]; ++k) cnt[m.es[k] + 1]++;
  for (int i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
  out.en_ptr = cnt;
  out.en.assign(cnt[N], 0);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int E = 0; E < n_ent; ++E)
    for (int64_t k = m.es_ptr[E]; k < m.es_ptr[E + 1]; ++k) out.en[fill[m.es[k]]++] = E;
  out.elem_pdof.assign((size_t)N * 4, -1);
  for (int i = 0; i < N; ++i) out.elem_pdof[(size_t)4 * i] = m.part_col[i];
  out.elem_part.resize(N);
  std::vector<int> pc(n_parts_next, 0);
  for (int i = 0; i < N; ++i) {
    const int p = parent[i];
    if (p < 0 || p >= n_parts_next) return "part_parent: id out of range";
    out.elem_part[i] = p;
    pc[p]++;
  }
  for (int j = 0; j < n_parts_next; ++j)
    if (!pc[j]) return "coarse part " + std::to_string(j) + " has no fine part";
  out.n_parts = n_parts_next;
  // entity graph: E ~ F if some node of E is adjacent to some node of F
  std::vector<int64_t> ac(n_ent + 1, 0);
  for (int u : m.gamma_nodes) {
    const int E = m.node_ent[u];
    for (int64_t k = mesh.adj_ptr[u]; k < mesh.adj_ptr[u + 1]; ++k) {
      const int F = m.node_ent[mesh.adj[k]];
      if (F >= 0 && F != E) ac[E + 1]++;
    }
  }
  for (int E = 0; E < n_ent; ++E) ac[E + 1] += ac[E];
  RawVec<int> nb(ac[n_ent]);
  std::vector<int64_t> af(ac.begin(), ac.end() - 1);
  for (int u : m.gamma_nodes) {
    const int E = m.node_ent[u];
    for (int64_t k = mesh.adj_ptr[u]; k < mesh.adj_ptr[u + 1]; ++k) {
      const int F = m.node_ent[mesh.adj[k]];
      if (F >= 0 && F != E) nb[af[E]++] = F;
    }
  }
  sort_unique_segments(ac, nb);
  out.adj_ptr = std::move(ac);
  out.adj = std::move(nb);
  return "";
}

void coarse_pattern(const LevelMaps& m, std::vector<int64_t>& rowptr, std::vector<int>& col) {
  const int nc = m.n_coarse;
  const int nthreads = host_threads();
  // per-thread stamps: column j is already in row c when stamp[j] == c
  std::vector<std::vector<int>> stamps(nthreads);
  auto row_walk = [&](int t, int c, auto&& emit) {
    std::vector<int>& stamp = stamps[t];
    if (stamp.size() != (size_t)nc) stamp.assign(nc, -1);
    for (int64_t k = m.cp_ptr[c]; k < m.cp_ptr[c + 1]; ++k) {
      const int i = m.cp_part[k];
      for (int64_t q = m.pc_ptr[i]; q < m.pc_ptr[i + 1]; ++q) {
        const int j = m.pcols[q];
        if (stamp[j] != c) {
          stamp[j] = c;
          emit(j);
        }
      }
    }
  };
  rowptr.assign(nc + 1, 0);
  parallel_for(nc, nthreads, [&](int t, int c0, int c1) {
    for (int c = c0; c < c1; ++c) {
      int64_t cnt = 0;
      row_walk(t, c, [&](int) { ++cnt; });
      rowptr[c + 1] = cnt;
    }
  });
  for (int c = 0; c < nc; ++c) rowptr[c + 1] += rowptr[c];
  col.resize(rowptr[nc]);
  for (auto& st : stamps) std::fill(st.begin(), st.end(), -1);
  parallel_for(nc, nthreads, [&](int t, int c0, int c1) {
    for (int c = c0; c < c1; ++c) {
      int* out = col.data() + rowptr[c];
      int64_t q = 0;
      row_walk(t, c, [&](int j) { out[q++] = j; });
      std::sort(out, out + q);
    }
  });
}

std::string scatter_lists(const LevelMaps& m, int64_t n, bool additive, std::vector<int64_t>& sc_ptr,
                          std::vector<int>& sc_pos) {
  const int N = (int)m.dom_ptr.size() - 1;
  const int64_t total = m.dom_ptr[N];
  if (additive) {
    sc_ptr.assign(n + 1, 0);
    for (int64_t k = 0; k < total; ++k) sc_ptr[m.dom[k] + 1]++;
    for (int64_t g = 0; g < n; ++g) sc_ptr[g + 1] += sc_ptr[g];
    sc_pos.resize(total);
    std::vector<int64_t> fill(sc_ptr.begin(), sc_ptr.end() - 1);
    for (int64_t k = 0; k < total; ++k) sc_pos[fill[m.dom[k]]++] = (int)k;
    return "";
  }
  // restricted: the one position of g inside its owner's domain
  sc_ptr.clear();
  sc_pos.assign(n, -1);
  const int nthreads = host_threads();
  std::vector<int64_t> found(nthreads, 0);
  parallel_for(N, nthreads, [&](int t, int i0, int i1) {
    for (int i = i0; i < i1; ++i)
      for (int64_t k = m.dom_ptr[i]; k < m.dom_ptr[i + 1]; ++k) {
        const int g = m.dom[k];
        if (m.owner[g] == i) {
          sc_pos[g] = (int)k;
          ++found[t];
        }
      }
  });
  int64_t f = 0;
  for (int64_t c : found) f += c;
  if (f != n) return "some dof is not held by its owning part";
  return "";
}

}  // namespace gdsw
