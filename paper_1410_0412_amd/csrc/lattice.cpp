// Host-side sparse-lattice builder: enumeration, adjacency list, RIA runs and
// their per-wavefront encoding (declared in include/lbm_sparse.h).
//
// Sect. 1 and Sect. 4: only fluid nodes are stored, in the order fixed by an
// enumeration function, and every node keeps 18 four-byte neighbour indices
// (the rest direction is addressed directly). Sect. 4.1: a node whose access
// pattern equals the previous node's shifted by one needs no index load; such
// runs are stored run-length coded. Sect. 5.6: lexicographic sorting with a
// blocking factor B, or a space-filling curve, as enumeration.
//
// All tables are built in O(voxels) passes that run in parallel over node or
// voxel ranges; only the Morton order needs a sort (LSD radix on the keys).
// The adjacency list itself (72 B per node) is never stored: the lattice
// keeps the voxel-to-node map (4 B per voxel) and computes a node's 18
// entries when a table or a caller needs them, so a lattice that fills a
// 288 GB device can be built with a small fraction of that in host memory.

#include "common.hpp"

#include <algorithm>
#include <climits>
#include <cstring>
#include <exception>
#include <new>
#include <system_error>
#include <thread>
#include <vector>

using namespace lbm;

struct lbm_lattice {
  int32_t nx = 0, ny = 0, nz = 0;
  uint32_t periodic = 0;            // bit a: axis a periodic
  bool plain_lex = false;           // LS order without blocking
  int64_t N = 0, R = 0, W = 0;
  std::vector<int32_t> node_voxel;  // [N]
  std::vector<int32_t> node_of;     // [nx*ny*nz]: node of a voxel, -1 if solid
  std::vector<int32_t> run_start;   // [R+1]
  std::vector<int32_t> run_delta;   // [18][R]
  std::vector<uint64_t> head_bits;  // [W]
  std::vector<int32_t> run_base;    // [W]
  // per-direction runs; RD < 0 when their count does not fit int32
  int64_t RD = 0;
  std::vector<int32_t> dir_delta;   // [RD]
  std::vector<uint64_t> dir_bits;   // [W][18]
  std::vector<int32_t> dir_base;    // [W][18]
};

namespace {

// Pull direction vectors c_q, q = 0..18 (same order as the kernels use).
constexpr int kC[19][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

// Run body(lo, hi) over [0, n) in up to 32 contiguous ranges on threads.
// Ranges that get no thread (thread creation failed) run on the calling
// thread. Every thread is joined before the first exception of any range is
// rethrown.
template <class F>
void parallel_for(int64_t n, F&& body) {
  unsigned hw = std::thread::hardware_concurrency();
  int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 1, 32));
  if (n < (int64_t)1 << 16) nt = 1;
  if (nt == 1) {
    body(int64_t(0), n);
    return;
  }
  const int64_t chunk = (n + nt - 1) / nt;
  std::vector<std::exception_ptr> err((size_t)nt);
  std::vector<std::thread> th;
  th.reserve((size_t)nt);
  auto range = [&](int64_t t) {
    const int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
    try {
      if (lo < hi) body(lo, hi);
    } catch (...) {
      err[(size_t)t] = std::current_exception();
    }
  };
  int64_t t = 0;
  for (; t < nt; ++t) {
    try {
      th.emplace_back(range, t);
    } catch (const std::system_error&) {
      break;
    }
  }
  for (; t < nt; ++t) range(t);
  for (auto& x : th) x.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

inline uint64_t spread3(uint64_t v) {
  // place bit b of v at bit 3b (v < 2^21)
  v &= 0x1fffffULL;
  v = (v | (v << 32)) & 0x1f00000000ffffULL;
  v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
  v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
  v = (v | (v << 2)) & 0x1249249249249249ULL;
  return v;
}

// LSD radix sort of (key, voxel) pairs by the low key_bits bits of the key.
void radix_sort(std::vector<uint64_t>& key, std::vector<int32_t>& val, int key_bits) {
  std::vector<uint64_t> k2(key.size());
  std::vector<int32_t> v2(val.size());
  const int digit = 11;
  const uint64_t dmask = (1u << digit) - 1;
  for (int shift = 0; shift < key_bits; shift += digit) {
    std::vector<int64_t> count((1 << digit) + 1, 0);
    for (uint64_t k : key) count[((k >> shift) & dmask) + 1]++;
    for (int i = 0; i < (1 << digit); ++i) count[i + 1] += count[i];
    for (size_t i = 0; i < key.size(); ++i) {
      int64_t dst = count[(key[i] >> shift) & dmask]++;
      k2[dst] = key[i];
      v2[dst] = val[i];
    }
    key.swap(k2);
    val.swap(v2);
  }
}

// Hilbert index of (x, y, z) on the 2^bits cube (Skilling's transpose
// method): remove the excess rotations / reflections level by level, Gray
// encode, and read the transposed bits interleaved, x first in each triple.
uint64_t hilbert_key(uint32_t x, uint32_t y, uint32_t z, int bits) {
  uint32_t X[3] = {x, y, z};
  const uint32_t top = 1u << (bits - 1);
  for (uint32_t Qb = top; Qb > 1; Qb >>= 1) {
    const uint32_t P = Qb - 1;
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Qb) {
        X[0] ^= P;
      } else {
        const uint32_t t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  uint32_t t = 0;
  for (uint32_t Qb = top; Qb > 1; Qb >>= 1)
    if (X[2] & Qb) t ^= Qb - 1;
  for (int i = 0; i < 3; ++i) X[i] ^= t;
  uint64_t key = 0;
  for (int b = bits - 1; b >= 0; --b)
    for (int i = 0; i < 3; ++i) key = (key << 1) | ((X[i] >> b) & 1u);
  return key;
}

int enumerate(lbm_lattice* L, const uint8_t* solid, int32_t order, int32_t block) {
  const int64_t nx = L->nx, ny = L->ny, nz = L->nz;
  auto& out = L->node_voxel;
  const int64_t maxext = std::max(nx, std::max(ny, nz));
  {
    int64_t fluid = 0;
    for (int64_t v = 0; v < nx * ny * nz; ++v) fluid += solid[v] == 0;
    out.reserve((size_t)fluid);
  }
  if (order == LBM_ORDER_LEX) {
    const int64_t B = block;
    if (B <= 1 || B >= maxext) {
      for (int64_t v = 0; v < nx * ny * nz; ++v)
        if (!solid[v]) out.push_back((int32_t)v);
    } else {
      for (int64_t bx = 0; bx < nx; bx += B)
        for (int64_t by = 0; by < ny; by += B)
          for (int64_t bz = 0; bz < nz; bz += B)
            for (int64_t x = bx; x < std::min(nx, bx + B); ++x)
              for (int64_t y = by; y < std::min(ny, by + B); ++y)
                for (int64_t z = bz; z < std::min(nz, bz + B); ++z) {
                  int64_t v = (x * ny + y) * nz + z;
                  if (!solid[v]) out.push_back((int32_t)v);
                }
    }
    return LBM_OK;
  }
  if (order == LBM_ORDER_MORTON) {
    if (maxext > (1 << 21)) return fail(LBM_ERANGE, "Morton order needs extents <= 2^21");
    int bits = 0;
    while ((int64_t(1) << bits) < maxext) ++bits;
    std::vector<uint64_t> keys;
    for (int64_t v = 0; v < nx * ny * nz; ++v) {
      if (solid[v]) continue;
      uint64_t x = v / (ny * nz), y = (v / nz) % ny, z = v % nz;
      keys.push_back((spread3(x) << 2) | (spread3(y) << 1) | spread3(z));
      out.push_back((int32_t)v);
    }
    radix_sort(keys, out, std::max(1, 3 * bits));
    return LBM_OK;
  }
  if (order == LBM_ORDER_HILBERT || order == LBM_ORDER_HILBERT_LS) {
    if (maxext > (1 << 21)) return fail(LBM_ERANGE, "Hilbert order needs extents <= 2^21");
    int bits = 1;
    while ((int64_t(1) << bits) < maxext) ++bits;
    std::vector<uint64_t> keys;
    for (int64_t v = 0; v < nx * ny * nz; ++v) {
      if (solid[v]) continue;
      keys.push_back(hilbert_key((uint32_t)(v / (ny * nz)), (uint32_t)((v / nz) % ny), (uint32_t)(v % nz), bits));
      out.push_back((int32_t)v);
    }
    radix_sort(keys, out, 3 * bits);
    if (order == LBM_ORDER_HILBERT_LS) {
      // two-stage renumbering (Sect. 6.1): partitions are contiguous chunks
      // of the curve, each re-enumerated lexicographically
      const int64_t parts = std::max<int32_t>(block, 1);
      const int64_t n = (int64_t)out.size();
      const int64_t chunk = n ? (n + parts - 1) / parts : 1;
      for (int64_t a = 0; a < n; a += chunk) std::sort(out.begin() + a, out.begin() + std::min(n, a + chunk));
    }
    return LBM_OK;
  }
  return fail(LBM_EINVAL, "unknown order %d", order);
}

void build_node_map(lbm_lattice* L) {
  const int64_t V = (int64_t)L->nx * L->ny * L->nz;
  L->node_of.assign((size_t)V, -1);
  parallel_for(L->N, [&](int64_t lo, int64_t hi) {
    for (int64_t n = lo; n < hi; ++n) L->node_of[L->node_voxel[n]] = (int32_t)n;
  });
}

// Adjacency entry of node n for direction q = 1..18 (pull: the node at
// x_n - c_q, or -1 if that site is solid or outside a non-periodic axis).
inline int32_t neighbour(const lbm_lattice* L, int64_t n, int q) {
  const int64_t ext[3] = {L->nx, L->ny, L->nz};
  const int64_t v = L->node_voxel[n];
  const int64_t x[3] = {v / (ext[1] * ext[2]), (v / ext[2]) % ext[1], v % ext[2]};
  int64_t u[3];
  for (int a = 0; a < 3; ++a) {
    u[a] = x[a] - kC[q][a];
    if (u[a] < 0 || u[a] >= ext[a]) {
      if (!(L->periodic & (1u << a))) return -1;
      u[a] = (u[a] + ext[a]) % ext[a];
    }
  }
  return L->node_of[(u[0] * ext[1] + u[1]) * ext[2] + u[2]];
}

inline void adjacency_of(const lbm_lattice* L, int64_t n, int32_t (&a)[18]) {
  for (int q = 1; q < 19; ++q) a[q - 1] = neighbour(L, n, q);
}

// The run rule of Sect. 4.1 for one direction: node n continues the run of
// n - 1 when its entry is the previous one shifted by one, or both are solid.
inline bool continues(int32_t prev, int32_t cur) { return prev >= 0 ? cur == prev + 1 : cur < 0; }

// Per-direction run heads, then the paper's (joint) runs: a node heads a
// joint run exactly when it heads a run of at least one direction. Runs of
// direction q are numbered after those of directions 1..q-1.
void build_runs(lbm_lattice* L) {
  const int64_t N = L->N, W = (N + kWave - 1) / kWave;
  L->W = W;
  L->dir_bits.assign((size_t)(W * 18), 0);
  parallel_for(W, [&](int64_t lo, int64_t hi) {
    int32_t a[kWave + 1][18];
    for (int64_t w = lo; w < hi; ++w) {
      const int64_t n0 = w * kWave, n1 = std::min(N, n0 + kWave);
      // row 0 holds node n0 - 1 (none for the first wave)
      if (n0 > 0) adjacency_of(L, n0 - 1, a[0]);
      for (int64_t n = n0; n < n1; ++n) adjacency_of(L, n, a[n - n0 + 1]);
      for (int q = 0; q < 18; ++q) {
        uint64_t bits = 0;
        for (int64_t n = n0; n < n1; ++n) {
          const bool cont = n > 0 && continues(a[n - n0][q], a[n - n0 + 1][q]);
          if (!cont) bits |= (uint64_t)1 << (n - n0);
        }
        L->dir_bits[(size_t)w * 18 + q] = bits;
      }
    }
  });

  // joint runs
  L->head_bits.assign((size_t)W, 0);
  L->run_base.assign((size_t)W, 0);
  for (int64_t w = 0; w < W; ++w) {
    uint64_t h = 0;
    for (int q = 0; q < 18; ++q) h |= L->dir_bits[(size_t)w * 18 + q];
    L->head_bits[w] = h;
  }
  L->run_start.clear();
  int64_t heads_below = 0;
  for (int64_t w = 0; w < W; ++w) {
    L->run_base[w] = (int32_t)(heads_below - 1);
    uint64_t bits = L->head_bits[w];
    heads_below += __builtin_popcountll(bits);
    while (bits) {
      L->run_start.push_back((int32_t)(w * kWave + __builtin_ctzll(bits)));
      bits &= bits - 1;
    }
  }
  L->R = (int64_t)L->run_start.size();
  L->run_start.push_back((int32_t)N);
  const int64_t R = L->R;
  L->run_delta.assign((size_t)(18 * R), INT32_MIN);
  parallel_for(R, [&](int64_t lo, int64_t hi) {
    int32_t a[18];
    for (int64_t r = lo; r < hi; ++r) {
      const int64_t h = L->run_start[r];
      adjacency_of(L, h, a);
      for (int q = 0; q < 18; ++q) L->run_delta[(size_t)q * R + r] = a[q] >= 0 ? (int32_t)(a[q] - h) : INT32_MIN;
    }
  });

  // per-direction run bases and deltas
  L->dir_base.assign((size_t)(W * 18), 0);
  int64_t first = 0;
  for (int q = 0; q < 18; ++q) {
    int64_t below = 0;
    for (int64_t w = 0; w < W; ++w) {
      const int64_t base = first + below - 1;
      if (base > INT32_MAX) {
        L->RD = -1;
        L->dir_bits.clear();
        L->dir_base.clear();
        return;
      }
      L->dir_base[(size_t)w * 18 + q] = (int32_t)base;
      below += __builtin_popcountll(L->dir_bits[(size_t)w * 18 + q]);
    }
    first += below;
  }
  if (first > INT32_MAX) {
    L->RD = -1;
    L->dir_bits.clear();
    L->dir_base.clear();
    return;
  }
  L->RD = first;
  L->dir_delta.assign((size_t)first, INT32_MIN);
  parallel_for(W, [&](int64_t lo, int64_t hi) {
    for (int64_t w = lo; w < hi; ++w)
      for (int q = 0; q < 18; ++q) {
        uint64_t bits = L->dir_bits[(size_t)w * 18 + q];
        int64_t r = (int64_t)L->dir_base[(size_t)w * 18 + q];
        while (bits) {
          const int l = __builtin_ctzll(bits);
          bits &= bits - 1;
          const int64_t h = w * kWave + l;
          const int32_t a = neighbour(L, h, q + 1);
          L->dir_delta[(size_t)++r] = a >= 0 ? (int32_t)(a - h) : INT32_MIN;
        }
      }
  });
}

}  // namespace

extern "C" {

// The message of the last failing call of any part of the library on this
// thread (the solver's calls set it too).
const char* lbm_last_error(void) { return error_buffer(); }

int lbm_lattice_build(const uint8_t* solid, int32_t nx, int32_t ny, int32_t nz,
                      uint32_t periodic_mask, int32_t order, int32_t block, lbm_lattice** out) {
  clear_error();
  if (!solid || !out) return fail(LBM_EINVAL, "null pointer");
  *out = nullptr;
  if (nx <= 0 || ny <= 0 || nz <= 0) return fail(LBM_EINVAL, "extents must be positive");
  if (block < 0) return fail(LBM_EINVAL, "block must be >= 0");
  if (periodic_mask > 7u) return fail(LBM_EINVAL, "periodic_mask has bits above 2");
  if ((int64_t)nx * ny * nz > INT32_MAX) return fail(LBM_ERANGE, "voxel count exceeds 2^31-1");
  lbm_lattice* L = new (std::nothrow) lbm_lattice;
  if (!L) return fail(LBM_ENOMEM, "out of host memory");
  L->nx = nx;
  L->ny = ny;
  L->nz = nz;
  try {
    int rc = enumerate(L, solid, order, block);
    if (rc != LBM_OK) {
      delete L;
      return rc;
    }
    L->N = (int64_t)L->node_voxel.size();
    L->periodic = periodic_mask;
    L->plain_lex = order == LBM_ORDER_LEX && (block <= 1 || block >= std::max(nx, std::max(ny, nz)));
    build_node_map(L);
    build_runs(L);
  } catch (const std::bad_alloc&) {
    delete L;
    return fail(LBM_ENOMEM, "out of host memory building the lattice");
  } catch (const std::exception& e) {
    delete L;
    return fail(LBM_ENOMEM, "host resources exhausted building the lattice: %s", e.what());
  }
  *out = L;
  return LBM_OK;
}

int lbm_lattice_sizes(const lbm_lattice* L, int64_t* n_fluid, int64_t* n_runs, int64_t* n_waves) {
  clear_error();
  if (!L) return fail(LBM_EINVAL, "null lattice");
  if (n_fluid) *n_fluid = L->N;
  if (n_runs) *n_runs = L->R;
  if (n_waves) *n_waves = L->W;
  return LBM_OK;
}

int lbm_lattice_copy_nodes(const lbm_lattice* L, int32_t* node_voxel) {
  clear_error();
  if (!L || !node_voxel) return fail(LBM_EINVAL, "null pointer");
  if (L->N) std::memcpy(node_voxel, L->node_voxel.data(), sizeof(int32_t) * L->N);
  return LBM_OK;
}

int lbm_lattice_copy_adjacency(const lbm_lattice* L, int32_t* adj, int64_t ld) {
  clear_error();
  if (!L || !adj) return fail(LBM_EINVAL, "null pointer");
  if (ld < L->N) return fail(LBM_EINVAL, "ld < N");
  parallel_for(L->N, [&](int64_t lo, int64_t hi) {
    int32_t a[18];
    for (int64_t n = lo; n < hi; ++n) {
      adjacency_of(L, n, a);
      for (int q = 0; q < 18; ++q) adj[q * ld + n] = a[q];
    }
  });
  for (int q = 0; q < 18; ++q) std::fill(adj + q * ld + L->N, adj + (q + 1) * ld, -1);
  return LBM_OK;
}

int lbm_lattice_copy_runs(const lbm_lattice* L, int32_t* run_start) {
  clear_error();
  if (!L || !run_start) return fail(LBM_EINVAL, "null pointer");
  std::memcpy(run_start, L->run_start.data(), sizeof(int32_t) * (L->R + 1));
  return LBM_OK;
}

int lbm_lattice_copy_wave_tables(const lbm_lattice* L, int32_t* run_delta, int64_t ldr,
                                 uint64_t* head_bits, int32_t* run_base) {
  clear_error();
  if (!L) return fail(LBM_EINVAL, "null lattice");
  if (run_delta) {
    if (ldr < L->R) return fail(LBM_EINVAL, "ldr < R");
    for (int q = 0; q < 18; ++q) {
      if (L->R) std::memcpy(run_delta + q * ldr, L->run_delta.data() + q * L->R, sizeof(int32_t) * L->R);
      std::fill(run_delta + q * ldr + L->R, run_delta + (q + 1) * ldr, INT32_MIN);
    }
  }
  if (head_bits && L->W) std::memcpy(head_bits, L->head_bits.data(), sizeof(uint64_t) * L->W);
  if (run_base && L->W) std::memcpy(run_base, L->run_base.data(), sizeof(int32_t) * L->W);
  return LBM_OK;
}

int lbm_lattice_direction_runs(const lbm_lattice* L, int64_t* n_dir_runs) {
  clear_error();
  if (!L || !n_dir_runs) return fail(LBM_EINVAL, "null pointer");
  if (L->RD < 0) return fail(LBM_ERANGE, "per-direction run count exceeds 2^31-1");
  *n_dir_runs = L->RD;
  return LBM_OK;
}

int lbm_lattice_copy_direction_tables(const lbm_lattice* L, int32_t* dir_delta, uint64_t* dir_bits,
                                      int32_t* dir_base) {
  clear_error();
  if (!L) return fail(LBM_EINVAL, "null lattice");
  if (L->RD < 0) return fail(LBM_ERANGE, "per-direction run count exceeds 2^31-1");
  if (dir_delta && L->RD) std::memcpy(dir_delta, L->dir_delta.data(), sizeof(int32_t) * L->RD);
  if (dir_bits && L->W) std::memcpy(dir_bits, L->dir_bits.data(), sizeof(uint64_t) * 18 * L->W);
  if (dir_base && L->W) std::memcpy(dir_base, L->dir_base.data(), sizeof(int32_t) * 18 * L->W);
  return LBM_OK;
}

int lbm_lattice_band_schedule(const lbm_lattice* L, int32_t band_rows, int32_t* sched, int64_t* len) {
  clear_error();
  if (!L || !len) return fail(LBM_EINVAL, "null pointer");
  if (!L->plain_lex) return fail(LBM_EINVAL, "band schedules need LS order without blocking");
  if (band_rows <= 0 || band_rows % kXcds != 0)
    return fail(LBM_EINVAL, "band_rows must be a positive multiple of %d", (int)kXcds);
  const int64_t G = (L->N + kGroupNodes - 1) / kGroupNodes;
  const int64_t ny = L->ny, nz = L->nz;
  // a block belongs to the band, x-plane and XCD of its first node: XCD k
  // takes rows [k, k + 1) * band_rows / 8 of every band
  std::vector<int64_t> count((size_t)kXcds, 0);
  for (int64_t g = 0; g < G; ++g) {
    const int64_t v = L->node_voxel[g * kGroupNodes];
    const int64_t y = (v / nz) % ny;
    ++count[(size_t)(((y % band_rows) * kXcds) / band_rows)];
  }
  const int64_t per = *std::max_element(count.begin(), count.end());
  const int64_t need = per * kXcds;
  if (!sched) {
    *len = need;
    return LBM_OK;
  }
  if (*len < need) return fail(LBM_EINVAL, "the schedule needs %lld entries", (long long)need);
  // blocks in (band, x-plane, node) order, dealt to their XCD's list
  const int64_t nxp = L->nx;
  std::vector<int64_t> key((size_t)G);
  std::vector<int64_t> order((size_t)G);
  for (int64_t g = 0; g < G; ++g) {
    const int64_t v = L->node_voxel[g * kGroupNodes];
    const int64_t x = v / (ny * nz), y = (v / nz) % ny;
    key[(size_t)g] = (y / band_rows) * nxp + x;
    order[(size_t)g] = g;
  }
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return key[(size_t)a] < key[(size_t)b]; });
  std::vector<int64_t> next((size_t)kXcds, 0);
  std::fill(sched, sched + need, -1);
  for (int64_t i = 0; i < G; ++i) {
    const int64_t g = order[(size_t)i];
    const int64_t v = L->node_voxel[g * kGroupNodes];
    const int64_t k = (((v / nz) % ny % band_rows) * kXcds) / band_rows;
    sched[next[(size_t)k]++ * kXcds + k] = (int32_t)g;
  }
  *len = need;
  return LBM_OK;
}

void lbm_lattice_free(lbm_lattice* L) { delete L; }

}  // extern "C"
