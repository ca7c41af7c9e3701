// Seeded synthetic-input generators for the PageRank path (host C++, OpenMP).
//
// This module produces graphs and batch updates only. It holds none of the
// PageRank arithmetic: no rank, contribution or convergence computation lives
// here. Both the HIP library's tests/benchmarks and the CPU oracle's tests take
// their inputs from it.
//
// Conventions fixed by the paper (Sec. 3.1 and Sec. 5.1.3, "Dataset" and
// "Batch Generation"):
//   * every vertex carries exactly one self-loop, so there are no dead ends;
//   * a batch update is a set of deletions (existing non-self-loop edges) and
//     insertions (edges not present), the vertex set is fixed;
//   * vertex IDs are 32-bit integers.
//
// Random numbers come from SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast
// splittable pseudorandom number generators", OOPSLA 2014), used as a
// counter-based generator: draw j of stream i is mix64(key(i) + j * GOLDEN),
// so every result is independent of the thread count.
//
// All entry points are extern "C" for ctypes; arrays are caller-owned host
// memory.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_set>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ULL;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Counter-based stream: the j-th draw of stream `id` under `seed`.
struct Stream {
  uint64_t state;
  Stream(uint64_t seed, uint64_t id) : state(mix64(mix64(seed) ^ mix64(id + GOLDEN))) {}
  inline uint64_t next() { state += GOLDEN; return mix64(state); }
  // uniform double in [0, 1) with 53 random bits
  inline double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  // uniform integer in [0, bound), bound > 0 (Lemire's multiply-shift, with rejection)
  inline uint64_t below(uint64_t bound) {
    for (;;) {
      uint64_t x = next();
      __uint128_t p = (__uint128_t)x * bound;
      uint64_t lo = (uint64_t)p;
      if (lo >= bound || lo >= (-bound) % bound) return (uint64_t)(p >> 64);
    }
  }
};

// A seeded bijection on [0, 2^bits): rounds of odd multiply, add, xor-shift.
struct Scrambler {
  int bits; uint64_t mask; uint64_t mul[3], add[3];
  Scrambler(int b, uint64_t seed) : bits(b) {
    mask = (b >= 64) ? ~0ULL : ((1ULL << b) - 1);
    Stream s(seed, 0x5C4A3B1EULL);
    for (int r = 0; r < 3; ++r) { mul[r] = s.next() | 1ULL; add[r] = s.next(); }
  }
  inline uint64_t operator()(uint64_t x) const {
    if (bits == 0) return 0;
    int sh = bits / 2 + 1;
    for (int r = 0; r < 3; ++r) {
      x = (x * mul[r] + add[r]) & mask;
      if (sh < bits) x ^= (x >> sh);
    }
    return x & mask;
  }
};

inline uint64_t pack(uint32_t hi, uint32_t lo) { return ((uint64_t)hi << 32) | lo; }

template <class T>
void exclusive_scan_inplace(T *a, int64_t n) {  // a[n] receives the total
  T run = 0;
  for (int64_t i = 0; i < n; ++i) { T t = a[i]; a[i] = run; run += t; }
  a[n] = run;
}

}  // namespace

extern "C" {

// R-MAT edges (Chakrabarti, Zhan, Faloutsos 2004), Graph500 style: for edge i,
// `scale` quadrant choices from the most significant bit down with
// probabilities (a, b, c, 1-a-b-c) for (src bit, dst bit) = (0,0), (0,1),
// (1,0), (1,1). If `scramble`, both endpoints pass through one seeded
// bijection of [0, 2^scale). Endpoints >= n are marked -1 (rejected) so that
// non-power-of-two vertex counts are possible.
void gg_rmat(int scale, int64_t n_edges, int32_t n, double a, double b, double c,
             uint64_t seed, int scramble, int32_t *src, int32_t *dst) {
  Scrambler scr(scale, seed ^ 0xA5A5A5A5ULL);
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_edges; ++i) {
    Stream s(seed, (uint64_t)i);
    uint64_t u = 0, v = 0;
    for (int lvl = 0; lvl < scale; lvl += 2) {
      uint64_t x = s.next();
      for (int k = 0; k < 2 && lvl + k < scale; ++k) {
        double p = (double)((k == 0 ? (x >> 32) : (x & 0xFFFFFFFFULL))) * (1.0 / 4294967296.0);
        int sb, db;
        if (p < a) { sb = 0; db = 0; }
        else if (p < ab) { sb = 0; db = 1; }
        else if (p < abc) { sb = 1; db = 0; }
        else { sb = 1; db = 1; }
        u = (u << 1) | (uint64_t)sb;
        v = (v << 1) | (uint64_t)db;
      }
    }
    if (scramble) { u = scr(u); v = scr(v); }
    bool ok = (u < (uint64_t)n) && (v < (uint64_t)n);
    src[i] = ok ? (int32_t)u : -1;
    dst[i] = ok ? (int32_t)v : -1;
  }
}

// Canonical graph from a raw edge list: edges with a negative endpoint are
// dropped, duplicates removed, one self-loop added per vertex, and both CSR
// views are built:
//   out CSR (G):  out_offsets[n+1], out_targets[m]; each row ascending;
//   in  CSR (G'): in_offsets[n+1],  in_sources[m];  each row ascending.
// Capacity of out_targets / in_sources must be >= e + n. Returns m.
int64_t gg_build(int32_t n, int64_t e, const int32_t *src, const int32_t *dst,
                 int32_t *out_offsets, int32_t *out_targets,
                 int32_t *in_offsets, int32_t *in_sources) {
  if (n <= 0) return -1;
  int nb_bits = 0;
  while ((1LL << nb_bits) < n) ++nb_bits;
  const int kb = std::min(nb_bits, 10);
  const int shift = nb_bits - kb;
  const int nbuckets = 1 << kb;
  const int nt = omp_get_max_threads();

  // ---- pass 1: scatter packed (src,dst) into src-range buckets (stable per thread)
  std::vector<int64_t> hist((size_t)nt * nbuckets, 0);
  std::vector<uint64_t> keys((size_t)e);
#pragma omp parallel num_threads(nt)
  {
    int t = omp_get_thread_num();
    int64_t lo = e * t / nt, hi = e * (t + 1) / nt;
    int64_t *h = &hist[(size_t)t * nbuckets];
    for (int64_t i = lo; i < hi; ++i)
      if (src[i] >= 0 && dst[i] >= 0) h[src[i] >> shift]++;
  }
  std::vector<int64_t> boff((size_t)nbuckets + 1, 0);
  {
    int64_t run = 0;
    for (int bkt = 0; bkt < nbuckets; ++bkt) {
      boff[bkt] = run;
      for (int t = 0; t < nt; ++t) {
        int64_t c = hist[(size_t)t * nbuckets + bkt];
        hist[(size_t)t * nbuckets + bkt] = run;
        run += c;
      }
    }
    boff[nbuckets] = run;
  }
#pragma omp parallel num_threads(nt)
  {
    int t = omp_get_thread_num();
    int64_t lo = e * t / nt, hi = e * (t + 1) / nt;
    int64_t *h = &hist[(size_t)t * nbuckets];
    for (int64_t i = lo; i < hi; ++i)
      if (src[i] >= 0 && dst[i] >= 0) keys[h[src[i] >> shift]++] = pack((uint32_t)src[i], (uint32_t)dst[i]);
  }

  // ---- pass 2: per bucket sort, dedupe, merge in self-loops; row degrees
  std::vector<int32_t> deg((size_t)n + 1, 0);
  std::vector<std::vector<int32_t>> btargets(nbuckets);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
  for (int bkt = 0; bkt < nbuckets; ++bkt) {
    int64_t lo = boff[bkt], hi = boff[bkt + 1];
    std::sort(keys.begin() + lo, keys.begin() + hi);
    int64_t r0 = (int64_t)bkt << shift, r1 = std::min<int64_t>((int64_t)(bkt + 1) << shift, n);
    if (r0 >= n) continue;
    std::vector<int32_t> &out = btargets[bkt];
    out.reserve((size_t)(hi - lo) + (size_t)(r1 - r0));
    int64_t p = lo;
    for (int64_t v = r0; v < r1; ++v) {
      size_t start = out.size();
      bool self_done = false;
      int64_t last = -1;
      while (p < hi && (int64_t)(keys[p] >> 32) == v) {
        int64_t w = (int64_t)(keys[p] & 0xFFFFFFFFULL);
        ++p;
        if (w == last) continue;
        if (!self_done && w >= v) {
          if (w != v) out.push_back((int32_t)v);
          self_done = true;
        }
        out.push_back((int32_t)w);
        last = w;
      }
      if (!self_done) out.push_back((int32_t)v);
      deg[v] = (int32_t)(out.size() - start);
    }
  }
  // out_offsets
  {
    int64_t run = 0;
    for (int64_t v = 0; v < n; ++v) { out_offsets[v] = (int32_t)run; run += deg[v]; }
    out_offsets[n] = (int32_t)run;
  }
  const int64_t m = out_offsets[n];
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
  for (int bkt = 0; bkt < nbuckets; ++bkt) {
    int64_t r0 = (int64_t)bkt << shift;
    if (r0 >= n) continue;
    const std::vector<int32_t> &out = btargets[bkt];
    if (!out.empty()) std::memcpy(out_targets + out_offsets[r0], out.data(), out.size() * sizeof(int32_t));
  }
  btargets.clear();
  btargets.shrink_to_fit();

  // ---- pass 3: transpose. Threads own contiguous source-row ranges, so the
  // scatter into dst-range buckets keeps ascending source order per bucket.
  std::fill(hist.begin(), hist.end(), 0);
  keys.resize((size_t)m);
#pragma omp parallel num_threads(nt)
  {
    int t = omp_get_thread_num();
    int64_t v0 = (int64_t)n * t / nt, v1 = (int64_t)n * (t + 1) / nt;
    int64_t *h = &hist[(size_t)t * nbuckets];
    for (int64_t i = out_offsets[v0]; i < out_offsets[v1]; ++i) h[out_targets[i] >> shift]++;
  }
  {
    int64_t run = 0;
    for (int bkt = 0; bkt < nbuckets; ++bkt) {
      boff[bkt] = run;
      for (int t = 0; t < nt; ++t) {
        int64_t c = hist[(size_t)t * nbuckets + bkt];
        hist[(size_t)t * nbuckets + bkt] = run;
        run += c;
      }
    }
    boff[nbuckets] = run;
  }
#pragma omp parallel num_threads(nt)
  {
    int t = omp_get_thread_num();
    int64_t v0 = (int64_t)n * t / nt, v1 = (int64_t)n * (t + 1) / nt;
    int64_t *h = &hist[(size_t)t * nbuckets];
    for (int64_t u = v0; u < v1; ++u)
      for (int64_t i = out_offsets[u]; i < out_offsets[u + 1]; ++i) {
        int32_t w = out_targets[i];
        keys[h[w >> shift]++] = pack((uint32_t)w, (uint32_t)u);
      }
  }
  std::fill(deg.begin(), deg.end(), 0);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
  for (int bkt = 0; bkt < nbuckets; ++bkt) {
    int64_t lo = boff[bkt], hi = boff[bkt + 1];
    // entries are grouped by thread and ascending in source within a thread;
    // a stable sort by destination keeps sources ascending per row.
    std::stable_sort(keys.begin() + lo, keys.begin() + hi,
                     [](uint64_t x, uint64_t y) { return (x >> 32) < (y >> 32); });
    for (int64_t i = lo; i < hi; ++i) deg[keys[i] >> 32]++;
  }
  {
    int64_t run = 0;
    for (int64_t v = 0; v < n; ++v) { in_offsets[v] = (int32_t)run; run += deg[v]; }
    in_offsets[n] = (int32_t)run;
  }
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
  for (int bkt = 0; bkt < nbuckets; ++bkt) {
    int64_t lo = boff[bkt], hi = boff[bkt + 1];
    if (lo == hi) continue;
    int64_t v = (int64_t)(keys[lo] >> 32);
    int64_t pos = in_offsets[v];
    for (int64_t i = lo; i < hi; ++i) in_sources[pos++] = (int32_t)(keys[i] & 0xFFFFFFFFULL);
  }
  return m;
}

// Expand an out-CSR into a (src, dst) edge list in row order.
void gg_csr_to_edges(int32_t n, const int32_t *offsets, const int32_t *targets,
                     int32_t *src, int32_t *dst) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t u = 0; u < n; ++u)
    for (int64_t i = offsets[u]; i < offsets[u + 1]; ++i) { src[i] = (int32_t)u; dst[i] = targets[i]; }
}

static bool has_edge(const int32_t *off, const int32_t *tgt, int32_t u, int32_t v) {
  return std::binary_search(tgt + off[u], tgt + off[u + 1], v);
}

// A random batch update on the canonical graph given by its out-CSR
// (paper Sec. 5.1.4, "Batch Generation"): n_ins insertions of uniformly
// random vertex pairs (u != v) that are not edges and are pairwise distinct,
// and n_del deletions drawn uniformly without replacement from the existing
// non-self-loop edges. Returns 0, or -1 if the graph cannot supply them.
int gg_random_batch(int32_t n, const int32_t *out_offsets, const int32_t *out_targets,
                    int64_t n_del, int64_t n_ins, uint64_t seed,
                    int32_t *del_src, int32_t *del_dst, int32_t *ins_src, int32_t *ins_dst) {
  const int64_t m = out_offsets[n];
  if (m - n < n_del) return -1;
  if ((double)n * (double)(n - 1) - (double)(m - n) < (double)n_ins) return -1;
  Stream s(seed, 0xBA7C4ULL);
  std::unordered_set<uint64_t> seen;
  seen.reserve((size_t)(n_ins + n_del) * 2 + 16);
  for (int64_t k = 0; k < n_ins;) {
    int32_t u = (int32_t)s.below((uint64_t)n), v = (int32_t)s.below((uint64_t)n);
    if (u == v || has_edge(out_offsets, out_targets, u, v)) continue;
    if (!seen.insert(pack((uint32_t)u, (uint32_t)v)).second) continue;
    ins_src[k] = u; ins_dst[k] = v; ++k;
  }
  seen.clear();
  // map a uniform edge index to its source row by binary search on offsets
  for (int64_t k = 0; k < n_del;) {
    int64_t e = (int64_t)s.below((uint64_t)m);
    const int32_t *it = std::upper_bound(out_offsets, out_offsets + n + 1, (int32_t)e);
    int32_t u = (int32_t)(it - out_offsets - 1);
    int32_t v = out_targets[e];
    if (u == v) continue;
    if (!seen.insert(pack((uint32_t)u, (uint32_t)v)).second) continue;
    del_src[k] = u; del_dst[k] = v; ++k;
  }
  return 0;
}

// Insertions of a temporal batch as a set difference: the unique pairs
// (src[i], dst[i]) with src != dst that are not edges of the graph, in order
// of first occurrence. Returns their number (written to ins_src/ins_dst).
int64_t gg_new_pairs(int32_t n, const int32_t *out_offsets, const int32_t *out_targets,
                     int64_t k, const int32_t *src, const int32_t *dst, int32_t *ins_src,
                     int32_t *ins_dst) {
  std::unordered_set<uint64_t> seen;
  seen.reserve((size_t)k * 2 + 16);
  int64_t c = 0;
  for (int64_t i = 0; i < k; ++i) {
    const int32_t u = src[i], v = dst[i];
    if (u < 0 || v < 0 || u >= n || v >= n || u == v) continue;
    if (has_edge(out_offsets, out_targets, u, v)) continue;
    if (!seen.insert(pack((uint32_t)u, (uint32_t)v)).second) continue;
    ins_src[c] = u;
    ins_dst[c] = v;
    ++c;
  }
  return c;
}

// Apply a batch to one CSR view (rows keyed by `row`, entries `col`): removes
// each (row, col) deletion and inserts each insertion, keeping rows sorted.
// The batch must be normalised (deletions present, insertions absent).
// new_cols capacity >= m + n_ins. Returns the new edge count or -1 if a
// deletion was not found or an insertion already existed.
int64_t gg_apply_view(int32_t n, const int32_t *offsets, const int32_t *cols,
                      int64_t n_del, const int32_t *del_row, const int32_t *del_col,
                      int64_t n_ins, const int32_t *ins_row, const int32_t *ins_col,
                      int32_t *new_offsets, int32_t *new_cols) {
  std::vector<uint64_t> dk((size_t)n_del), ik((size_t)n_ins);
  for (int64_t i = 0; i < n_del; ++i) dk[i] = pack((uint32_t)del_row[i], (uint32_t)del_col[i]);
  for (int64_t i = 0; i < n_ins; ++i) ik[i] = pack((uint32_t)ins_row[i], (uint32_t)ins_col[i]);
  std::sort(dk.begin(), dk.end());
  std::sort(ik.begin(), ik.end());
  std::vector<int64_t> dstart((size_t)n + 1, 0), istart((size_t)n + 1, 0);
  for (auto k : dk) dstart[(k >> 32) + 1]++;
  for (auto k : ik) istart[(k >> 32) + 1]++;
  for (int64_t v = 0; v < n; ++v) { dstart[v + 1] += dstart[v]; istart[v + 1] += istart[v]; }
  std::vector<int32_t> deg((size_t)n + 1);
  for (int64_t v = 0; v < n; ++v)
    deg[v] = (offsets[v + 1] - offsets[v]) - (int32_t)(dstart[v + 1] - dstart[v]) +
             (int32_t)(istart[v + 1] - istart[v]);
  {
    int64_t run = 0;
    for (int64_t v = 0; v < n; ++v) { new_offsets[v] = (int32_t)run; run += deg[v]; }
    new_offsets[n] = (int32_t)run;
  }
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1024) reduction(| : bad)
  for (int64_t v = 0; v < n; ++v) {
    int64_t p = offsets[v], pe = offsets[v + 1];
    int64_t d = dstart[v], de = dstart[v + 1];
    int64_t q = istart[v], qe = istart[v + 1];
    int64_t w = new_offsets[v], we = new_offsets[v + 1];
    auto ins_at = [&](int64_t i) { return (int32_t)(ik[i] & 0xFFFFFFFFULL); };
    auto del_at = [&](int64_t i) { return (int32_t)(dk[i] & 0xFFFFFFFFULL); };
    auto emit = [&](int32_t c) { if (w < we) new_cols[w] = c; else bad = 1; ++w; };
    while (p < pe) {
      int32_t a = cols[p++];
      while (q < qe && ins_at(q) < a) emit(ins_at(q++));
      if (q < qe && ins_at(q) == a) { bad = 1; ++q; }     // insertion of an existing edge
      while (d < de && del_at(d) < a) { bad = 1; ++d; }   // deletion of a missing edge
      if (d < de && del_at(d) == a) { ++d; continue; }
      emit(a);
    }
    while (q < qe) emit(ins_at(q++));
    if (d != de || w != we) bad = 1;
  }
  return bad ? -1 : (int64_t)new_offsets[n];
}

// Preferential-attachment temporal edge stream. Vertex i >= 1 arrives in ID
// order and emits k_i out-edges, k_i drawn from the discrete power law
// P(k) ~ k^-gamma on [k_min, k_max] (exact inverse CDF over a table); each
// target is drawn with replacement from vertices j < i with weight
// deg_in(j) + deg_out(j) + 1 (degrees counted over events emitted so far).
// Stops after exactly n_events events (src, dst); if all n vertices have
// arrived first, further events come from uniformly drawn sources with the
// same target rule. Repeated pairs are temporal duplicates. Sequential by
// construction; a Fenwick tree holds the vertex weights. Returns the count.
int64_t gg_pa_temporal(int32_t n, int64_t n_events, double gamma, int32_t k_min, int32_t k_max,
                       uint64_t seed, int32_t *src, int32_t *dst) {
  if (n <= 1 || k_min < 1 || k_max < k_min) return -1;
  std::vector<double> cdf((size_t)(k_max - k_min + 1));
  {
    double run = 0.0;
    for (int64_t k = k_min; k <= k_max; ++k) { run += std::pow((double)k, -gamma); cdf[k - k_min] = run; }
    for (auto &c : cdf) c /= run;
  }
  std::vector<int64_t> tree((size_t)n + 1, 0);
  int64_t logn = 1;
  while ((logn << 1) <= n) logn <<= 1;
  auto add = [&](int64_t i, int64_t dv) { for (++i; i <= n; i += i & (-i)) tree[i] += dv; };
  auto find = [&](int64_t target) {  // smallest idx with prefix(idx+1) > target
    int64_t pos = 0;
    for (int64_t step = logn; step > 0; step >>= 1)
      if (pos + step <= n && tree[pos + step] <= target) { pos += step; target -= tree[pos]; }
    return pos;
  };
  Stream s(seed, 0x7E3AULL);
  int64_t total = 1, k = 0;
  add(0, 1);  // vertex 0 exists with weight deg 0 + 1
  for (int32_t i = 1; i < n && k < n_events; ++i) {
    double u = s.uniform();
    int64_t ki = k_min + (int64_t)(std::upper_bound(cdf.begin(), cdf.end(), u) - cdf.begin());
    if (ki > k_max) ki = k_max;
    for (int64_t j = 0; j < ki && k < n_events; ++j) {
      int64_t t = find((int64_t)s.below((uint64_t)total));
      src[k] = i; dst[k] = (int32_t)t; ++k;
      add(t, 1); ++total;  // the target gains one in-edge
    }
    add(i, 1 + ki); total += 1 + ki;  // vertex i joins with its out-degree + 1
  }
  while (k < n_events) {
    int32_t i = (int32_t)s.below((uint64_t)n);
    int64_t t = find((int64_t)s.below((uint64_t)total));
    src[k] = i; dst[k] = (int32_t)t; ++k;
    add(t, 1); add(i, 1); total += 2;
  }
  return k;
}

// Per-edge weight in (lo, hi], a pure function of (seed, u, v) so that both
// CSR views of one edge see one value.
void gg_edge_weights(int64_t m, const int32_t *u, const int32_t *v, uint64_t seed,
                     double lo, double hi, double *w) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    uint64_t h = mix64(mix64(seed) ^ pack((uint32_t)u[i], (uint32_t)v[i]));
    double x = (double)(h >> 11) * (1.0 / 9007199254740992.0);  // [0,1)
    w[i] = hi - (hi - lo) * x;                                   // (lo, hi]
  }
}

// k distinct uniform vertex IDs per set, `sets` sets, written row-major.
void gg_distinct_vertices(int32_t n, int32_t sets, int32_t k, uint64_t seed, int32_t *out) {
  for (int32_t q = 0; q < sets; ++q) {
    Stream s(seed, (uint64_t)q);
    std::unordered_set<int32_t> got;
    for (int32_t j = 0; j < k;) {
      int32_t v = (int32_t)s.below((uint64_t)n);
      if (got.insert(v).second) out[(int64_t)q * k + j++] = v;
    }
  }
}

// Uniform doubles in [0,1) for stream `seed`.
void gg_uniform(int64_t count, uint64_t seed, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) {
    Stream s(seed, (uint64_t)i);
    out[i] = s.uniform();
  }
}

}  // extern "C"
