// Host self-check of the sparse-lattice builder through the C ABI, built for
// the CPU with AddressSanitizer and UndefinedBehaviorSanitizer (a plain C++
// build of lattice.cpp, no device code). It builds lattices of small seeded
// masks under every periodicity, enumeration and a range of blocking factors,
// and the paper's empty 500x100x100 channel (Sect. 5.1), copies every table
// and checks what the tables must satisfy by their definitions:
//  * node_voxel lists each fluid voxel exactly once (Sect. 1: only fluid
//    nodes are stored);
//  * the adjacency entry of direction q at node n is the fluid node at
//    x_n - c_q, or -1 (Sect. 4), so following q and then its opposite
//    returns to n;
//  * runs (Sect. 4.1) are maximal: inside a run every entry of node n is the
//    entry of n-1 plus one (or both are -1), and at each run head some entry
//    breaks that rule;
//  * the wave tables and the per-direction tables give back the adjacency
//    list for every node and direction;
//  * the AA odd step's slot map (f_q of node n at slot (qbar, a_q(n)) if
//    that neighbour is fluid, else (q, n)) and the OS-NT pull map ((q,
//    a_q(n)) or (qbar, n)) are bijections on the 19 N slots: every slot is
//    read by exactly one (node, direction), so the in-place AA update has no
//    race and the pull step reads every stored value once;
//  * invalid arguments return the documented error codes.
// Usage: lattice_check [channel]   (exit status 0 when every check passes)

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lbm_sparse.h"

namespace {

constexpr int kC[19][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
constexpr int kOpp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

int g_failures = 0;

void expect(bool ok, const char* what, const char* ctx) {
  if (!ok) {
    if (g_failures < 20) std::fprintf(stderr, "FAIL %s [%s]\n", what, ctx);
    ++g_failures;
  }
}

// xorshift64*: seeded masks without the C library's rand()
struct Rng {
  uint64_t s;
  uint64_t next() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return s * 0x2545F4914F6CDD1DULL;
  }
};

void check_lattice(const std::vector<uint8_t>& mask, int nx, int ny, int nz, uint32_t per, int order,
                   int block, const char* ctx) {
  lbm_lattice* lat = nullptr;
  int rc = lbm_lattice_build(mask.data(), nx, ny, nz, per, order, block, &lat);
  expect(rc == LBM_OK && lat, "build", ctx);
  if (rc != LBM_OK) return;
  int64_t N = 0, R = 0, W = 0;
  expect(lbm_lattice_sizes(lat, &N, &R, &W) == LBM_OK, "sizes", ctx);
  const int64_t cells = (int64_t)nx * ny * nz;
  int64_t fluid = 0;
  for (uint8_t m : mask) fluid += m == 0;
  expect(N == fluid, "N equals the fluid voxel count", ctx);
  expect(W == (N + 63) / 64, "W = ceil(N/64)", ctx);

  std::vector<int32_t> nodes((size_t)N + 1, -7);
  expect(lbm_lattice_copy_nodes(lat, nodes.data()) == LBM_OK, "copy nodes", ctx);
  expect(nodes[(size_t)N] == -7, "copy nodes writes N entries", ctx);
  std::vector<int32_t> node_of((size_t)cells, -1);
  for (int64_t n = 0; n < N; ++n) {
    const int32_t v = nodes[(size_t)n];
    const bool in = v >= 0 && v < cells;
    expect(in && mask[(size_t)v] == 0, "node voxel is a fluid voxel", ctx);
    if (!in) continue;
    expect(node_of[(size_t)v] < 0, "each fluid voxel once", ctx);
    node_of[(size_t)v] = (int32_t)n;
  }

  const int64_t ld = N + 5;
  std::vector<int32_t> adj((size_t)(18 * ld));
  expect(lbm_lattice_copy_adjacency(lat, adj.data(), ld) == LBM_OK, "copy adjacency", ctx);
  const int dims[3] = {nx, ny, nz};
  for (int64_t n = 0; n < N; ++n) {
    const int32_t v = nodes[(size_t)n];
    const int p[3] = {(int)(v / ((int64_t)ny * nz)), (int)(v / nz % ny), (int)(v % nz)};
    for (int q = 1; q < 19; ++q) {
      int up[3];
      bool inside = true;
      for (int a = 0; a < 3; ++a) {
        up[a] = p[a] - kC[q][a];
        if (up[a] < 0 || up[a] >= dims[a]) {
          if (per >> a & 1)
            up[a] = (up[a] + dims[a]) % dims[a];
          else
            inside = false;
        }
      }
      int32_t want = -1;
      if (inside) want = node_of[(size_t)(((int64_t)up[0] * ny + up[1]) * nz + up[2])];
      const int32_t got = adj[(size_t)((q - 1) * ld + n)];
      expect(got == want, "adjacency entry is the upstream fluid node", ctx);
      if (got >= 0 && got < N)
        expect(adj[(size_t)((kOpp[q] - 1) * ld + got)] == (int32_t)n, "opposite entry leads back", ctx);
    }
    for (int q = 1; q < 19; ++q)
      for (int64_t c = N; c < ld; ++c) expect(adj[(size_t)((q - 1) * ld + c)] == -1, "padding columns -1", ctx);
  }

  // slot maps of the AA odd step and of the pull step: bijections on 19 N slots
  for (int map = 0; map < 2; ++map) {
    std::vector<uint8_t> hit((size_t)(19 * N), 0);
    bool ok = true;
    for (int64_t n = 0; n < N; ++n) {
      for (int q = 0; q < 19; ++q) {
        int64_t slot = n;  // direction 0: the node's own rest slot
        if (q > 0) {
          const int32_t a = adj[(size_t)((q - 1) * ld + n)];
          const int k = map == 0 ? (a >= 0 ? kOpp[q] : q) : (a >= 0 ? q : kOpp[q]);
          slot = (int64_t)k * N + (a >= 0 ? a : n);
        }
        if (slot < 0 || slot >= 19 * N || hit[(size_t)slot]++) ok = false;
      }
    }
    expect(ok, map == 0 ? "AA odd-step slot map is a bijection" : "pull map is a bijection", ctx);
  }

  std::vector<int32_t> start((size_t)R + 1);
  expect(lbm_lattice_copy_runs(lat, start.data()) == LBM_OK, "copy runs", ctx);
  expect(start[0] == 0 && start[(size_t)R] == N, "run starts span the nodes", ctx);
  auto shifted = [&](int64_t n, int q) {
    const int32_t a = adj[(size_t)((q - 1) * ld + n)], b = adj[(size_t)((q - 1) * ld + n - 1)];
    return (b >= 0 && a == b + 1) || (b < 0 && a < 0);
  };
  std::vector<uint8_t> head((size_t)N, 0);
  for (int64_t r = 0; r < R; ++r) {
    expect(start[(size_t)r] < start[(size_t)r + 1], "runs are not empty", ctx);
    if (start[(size_t)r] >= 0 && start[(size_t)r] < N) head[(size_t)start[(size_t)r]] = 1;
  }
  for (int64_t n = 1; n < N; ++n) {
    bool cont = true;
    for (int q = 1; q < 19; ++q) cont = cont && shifted(n, q);
    expect(cont == !head[(size_t)n], "runs are maximal", ctx);
  }

  const int64_t ldr = R + 3;
  std::vector<int32_t> delta((size_t)(18 * ldr));
  std::vector<uint64_t> bits((size_t)W);
  std::vector<int32_t> base((size_t)W);
  expect(lbm_lattice_copy_wave_tables(lat, delta.data(), ldr, bits.data(), base.data()) == LBM_OK, "wave tables",
         ctx);
  for (int64_t n = 0; n < N; ++n) {
    const int64_t w = n / 64;
    const int l = (int)(n % 64);
    const uint64_t upto = l == 63 ? ~0ULL : ((2ULL << l) - 1);
    const int64_t r = base[(size_t)w] + __builtin_popcountll(bits[(size_t)w] & upto);
    expect(r >= 0 && r < R, "run index in range", ctx);
    if (r < 0 || r >= R) continue;
    for (int q = 1; q < 19; ++q) {
      const int32_t d = delta[(size_t)((q - 1) * ldr + r)];
      const int32_t a = d == INT32_MIN ? -1 : (int32_t)(n + d);
      expect(a == adj[(size_t)((q - 1) * ld + n)], "wave tables give the adjacency", ctx);
    }
  }

  int64_t RD = 0;
  if (lbm_lattice_direction_runs(lat, &RD) == LBM_OK) {
    std::vector<int32_t> dd((size_t)RD);
    std::vector<uint64_t> db((size_t)(18 * W));
    std::vector<int32_t> dbase((size_t)(18 * W));
    expect(lbm_lattice_copy_direction_tables(lat, dd.data(), db.data(), dbase.data()) == LBM_OK,
           "direction tables", ctx);
    for (int64_t n = 0; n < N; ++n) {
      const int64_t w = n / 64;
      const int l = (int)(n % 64);
      const uint64_t upto = l == 63 ? ~0ULL : ((2ULL << l) - 1);
      for (int q = 1; q < 19; ++q) {
        const int64_t k = 18 * w + q - 1;
        const int64_t r = dbase[(size_t)k] + __builtin_popcountll(db[(size_t)k] & upto);
        expect(r >= 0 && r < RD, "direction run index in range", ctx);
        if (r < 0 || r >= RD) continue;
        const int32_t d = dd[(size_t)r];
        const int32_t a = d == INT32_MIN ? -1 : (int32_t)(n + d);
        expect(a == adj[(size_t)((q - 1) * ld + n)], "direction tables give the adjacency", ctx);
      }
    }
  }
  lbm_lattice_free(lat);
}

void check_errors() {
  const uint8_t m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  lbm_lattice* lat = nullptr;
  expect(lbm_lattice_build(nullptr, 2, 2, 2, 0, 0, 0, &lat) == LBM_EINVAL, "null mask", "errors");
  expect(lbm_lattice_build(m, 2, 2, 2, 0, 0, 0, nullptr) == LBM_EINVAL, "null out", "errors");
  expect(lbm_lattice_build(m, 0, 2, 2, 0, 0, 0, &lat) == LBM_EINVAL, "zero extent", "errors");
  expect(lbm_lattice_build(m, 2, -2, 2, 0, 0, 0, &lat) == LBM_EINVAL, "negative extent", "errors");
  expect(lbm_lattice_build(m, 2, 2, 2, 0, 0, -1, &lat) == LBM_EINVAL, "negative block", "errors");
  expect(lbm_lattice_build(m, 2, 2, 2, 0, 9, 0, &lat) == LBM_EINVAL, "unknown order", "errors");
  expect(lbm_lattice_build(m, 2, 2, 2, 8u, 0, 0, &lat) == LBM_EINVAL, "periodic bits above 2", "errors");
  expect(lbm_lattice_build(m, 65536, 65536, 2, 0, 0, 0, &lat) == LBM_ERANGE, "too many voxels", "errors");
  expect(*lbm_last_error() != 0, "error message", "errors");
  expect(lbm_lattice_sizes(nullptr, nullptr, nullptr, nullptr) == LBM_EINVAL, "null lattice", "errors");
}

}  // namespace

int main(int argc, char** argv) {
  check_errors();
  Rng rng{0x9E3779B97F4A7C15ULL};
  const int shapes[][3] = {{1, 1, 1}, {3, 4, 5}, {7, 5, 6}, {9, 8, 7}, {16, 3, 11}};
  const int orders[] = {LBM_ORDER_LEX, LBM_ORDER_MORTON, LBM_ORDER_HILBERT, LBM_ORDER_HILBERT_LS};
  const int blocks[] = {0, 1, 2, 3, 4, 64};
  char ctx[160];
  int cases = 0;
  for (const auto& sh : shapes) {
    const int nx = sh[0], ny = sh[1], nz = sh[2];
    for (int fill = 0; fill < 3; ++fill) {
      std::vector<uint8_t> mask((size_t)nx * ny * nz);
      for (auto& v : mask) v = fill == 0 ? 0 : (uint8_t)(rng.next() % (fill == 1 ? 5 : 2) == 0);
      for (uint32_t per = 0; per < 8; ++per)
        for (int order : orders)
          for (int block : blocks) {
            if (order == LBM_ORDER_MORTON || order == LBM_ORDER_HILBERT) {
              if (block != 0) continue;
            } else if (order == LBM_ORDER_HILBERT_LS && block == 0) {
              continue;
            }
            std::snprintf(ctx, sizeof ctx, "%dx%dx%d fill %d periodic %u order %d block %d", nx, ny, nz, fill,
                          per, order, block);
            check_lattice(mask, nx, ny, nz, per, order, block, ctx);
            ++cases;
          }
    }
  }
  if (argc > 1 && argv[1][0] == 'c') {
    // the paper's empty channel: one-voxel walls on the y and z faces
    const int nx = 500, ny = 100, nz = 100;
    std::vector<uint8_t> mask((size_t)nx * ny * nz, 0);
    for (int x = 0; x < nx; ++x)
      for (int y = 0; y < ny; ++y)
        for (int z = 0; z < nz; ++z)
          if (y == 0 || y == ny - 1 || z == 0 || z == nz - 1) mask[((size_t)x * ny + y) * nz + z] = 1;
    check_lattice(mask, nx, ny, nz, 1u, LBM_ORDER_LEX, 1, "channel 500x100x100, LS B=1");
    ++cases;
  }
  std::printf("lattice_check: %d lattices, %d failures\n", cases, g_failures);
  return g_failures == 0 ? 0 : 1;
}
