// lbm_run: a command-line driver of the C ABI (include/lbm_sparse.h).
//
// It builds the sparse lattice of a voxel mask, allocates every device buffer
// itself with the HIP runtime, runs a solver from the rest state and writes
// the PDFs f(t) in natural node order. Nothing but the C ABI and the HIP
// runtime is used, so the program shows the library driven without Python.
//
// usage: lbm_run MASK NX NY NZ PERIODIC ORDER BLOCK PATTERN INDEX PRECISION
//                TAU FX FY FZ STEPS OUT [BAND_ROWS]
//   MASK       file of NX*NY*NZ bytes in C order (x slowest); nonzero = solid
//   PERIODIC   bit mask of the periodic axes (1 = x, 2 = y, 4 = z)
//   ORDER      lex | morton | hilbert | hilbert_ls (BLOCK: blocking factor,
//              or the number of chunks of hilbert_ls)
//   PATTERN    aa | osnt
//   INDEX      adjacency | runs | direction
//   PRECISION  f64 | f32 | f16
//   BAND_ROWS  optional: launch the AA odd step in the band schedule with
//              this many rows per band (lbm_lattice_band_schedule); 0 or
//              absent: the default order
// OUT receives int64 N, int32 node_voxel[N] and double f[19][N] (f(STEPS),
// direction-major). One line on stdout reports N, the runs and the totals
// (mass, jx, jy, jz). Exit status 0 on success, 1 on any error.

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_sparse.h"

namespace {

[[noreturn]] void die(const char* what, const char* detail) {
  std::fprintf(stderr, "lbm_run: %s: %s\n", what, detail);
  std::exit(1);
}

void check(int rc, const char* what) {
  if (rc != LBM_OK) die(what, lbm_last_error());
}

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) die(what, hipGetErrorString(e));
}

// Device buffer owned by this program; freed at the end of main.
struct DeviceBuffer {
  void* p = nullptr;
  void alloc(size_t bytes, const char* what) { check_hip(hipMalloc(&p, bytes ? bytes : 8), what); }
  template <class T>
  void upload(const std::vector<T>& h, const char* what) {
    alloc(h.size() * sizeof(T), what);
    if (!h.empty()) check_hip(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), what);
  }
  ~DeviceBuffer() {
    if (p) (void)hipFree(p);
  }
};

int64_t round_up(int64_t n, int64_t m) { return (n + m - 1) / m * m; }

int pick(const char* s, const char* const* names, int count, const char* what) {
  for (int i = 0; i < count; ++i)
    if (std::strcmp(s, names[i]) == 0) return i;
  die(what, s);
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 17 && argc != 18) {
    std::fprintf(stderr,
                 "usage: %s MASK NX NY NZ PERIODIC ORDER BLOCK PATTERN INDEX PRECISION TAU FX FY FZ STEPS OUT"
                 " [BAND_ROWS]\n",
                 argv[0]);
    return 1;
  }
  const int32_t band_rows = argc == 18 ? std::atoi(argv[17]) : 0;
  const int32_t nx = std::atoi(argv[2]), ny = std::atoi(argv[3]), nz = std::atoi(argv[4]);
  const uint32_t periodic = (uint32_t)std::atoi(argv[5]);
  static const char* const kOrders[] = {"lex", "morton", "hilbert", "hilbert_ls"};
  static const int kOrderIds[] = {LBM_ORDER_LEX, LBM_ORDER_MORTON, LBM_ORDER_HILBERT, LBM_ORDER_HILBERT_LS};
  const int order = kOrderIds[pick(argv[6], kOrders, 4, "unknown order")];
  const int32_t block = std::atoi(argv[7]);
  static const char* const kPatterns[] = {"aa", "osnt"};
  const int pattern = pick(argv[8], kPatterns, 2, "unknown pattern") == 0 ? LBM_PATTERN_AA : LBM_PATTERN_OSNT;
  static const char* const kIndex[] = {"adjacency", "runs", "direction"};
  static const int kIndexIds[] = {LBM_INDEX_ADJ, LBM_INDEX_RUNS, LBM_INDEX_DIRECTION_RUNS};
  const int index = kIndexIds[pick(argv[9], kIndex, 3, "unknown index source")];
  static const char* const kPrec[] = {"f64", "f32", "f16"};
  static const int kPrecIds[] = {LBM_F64, LBM_F32, LBM_F16};
  const int prec_i = pick(argv[10], kPrec, 3, "unknown precision");
  const double tau = std::atof(argv[11]);
  const double force[3] = {std::atof(argv[12]), std::atof(argv[13]), std::atof(argv[14])};
  const int64_t steps = std::atoll(argv[15]);
  if (nx <= 0 || ny <= 0 || nz <= 0) die("bad extents", argv[2]);

  // voxel mask
  const size_t cells = (size_t)nx * (size_t)ny * (size_t)nz;
  std::vector<uint8_t> mask(cells);
  FILE* fm = std::fopen(argv[1], "rb");
  if (!fm) die("cannot open mask", argv[1]);
  const size_t got = std::fread(mask.data(), 1, cells, fm);
  const bool extra = std::fgetc(fm) != EOF;
  std::fclose(fm);
  if (got != cells || extra) die("mask size is not NX*NY*NZ bytes", argv[1]);

  // host lattice and its tables
  lbm_lattice* lat = nullptr;
  check(lbm_lattice_build(mask.data(), nx, ny, nz, periodic, order, block, &lat), "lattice build");
  int64_t N = 0, R = 0, W = 0;
  check(lbm_lattice_sizes(lat, &N, &R, &W), "lattice sizes");
  std::vector<int32_t> node_voxel((size_t)N);
  check(lbm_lattice_copy_nodes(lat, node_voxel.data()), "node list");

  lbm_params p;
  std::memset(&p, 0, sizeof p);
  p.tau = tau;
  for (int a = 0; a < 3; ++a) p.force[a] = force[a];
  p.rho0 = 1.0;
  p.pattern = pattern;
  p.ria = index;
  p.precision = kPrecIds[prec_i];
  p.n_fluid = N;
  p.ldf = round_up(N > 0 ? N : 1, 64);
  p.f16_scale_log2 = 10;
  p.collision = LBM_BGK;

  // grid and workspace sizes as the library states them
  int64_t grid_bytes = 0, ws_bytes = 0;
  check(lbm_required_bytes(&p, &grid_bytes, &ws_bytes), "required bytes");
  DeviceBuffer grid[2], adj, delta, bits, base, ws, f_dev, tot_dev, sched_dev;
  grid[0].alloc((size_t)grid_bytes, "grid allocation");
  if (pattern == LBM_PATTERN_OSNT) grid[1].alloc(grid_bytes, "grid allocation");

  int64_t runs_used = 0;
  if (index == LBM_INDEX_ADJ) {
    p.lda = round_up(N > 0 ? N : 1, 64);
    std::vector<int32_t> h((size_t)(18 * p.lda));
    check(lbm_lattice_copy_adjacency(lat, h.data(), p.lda), "adjacency list");
    adj.upload(h, "adjacency upload");
  } else if (index == LBM_INDEX_RUNS) {
    p.ldr = round_up(R > 0 ? R : 1, 64);
    p.n_runs = R;
    runs_used = R;
    std::vector<int32_t> d((size_t)(18 * p.ldr)), b0((size_t)W);
    std::vector<uint64_t> b1((size_t)W);
    check(lbm_lattice_copy_wave_tables(lat, d.data(), p.ldr, b1.data(), b0.data()), "wave tables");
    delta.upload(d, "run table upload");
    bits.upload(b1, "run table upload");
    base.upload(b0, "run table upload");
  } else {
    int64_t RD = 0;
    check(lbm_lattice_direction_runs(lat, &RD), "per-direction runs");
    p.n_runs = RD;
    runs_used = RD;
    std::vector<int32_t> d((size_t)RD), b0((size_t)(18 * W));
    std::vector<uint64_t> b1((size_t)(18 * W));
    check(lbm_lattice_copy_direction_tables(lat, d.data(), b1.data(), b0.data()), "per-direction tables");
    delta.upload(d, "run table upload");
    bits.upload(b1, "run table upload");
    base.upload(b0, "run table upload");
  }
  // the odd step's band schedule, built from the lattice before it is freed
  std::vector<int32_t> sched;
  if (band_rows > 0) {
    int64_t len = 0;
    check(lbm_lattice_band_schedule(lat, band_rows, nullptr, &len), "band schedule");
    sched.resize((size_t)len);
    check(lbm_lattice_band_schedule(lat, band_rows, sched.data(), &len), "band schedule");
  }
  lbm_lattice_free(lat);

  lbm_buffers b;
  std::memset(&b, 0, sizeof b);
  b.pdf[0] = grid[0].p;
  b.pdf[1] = grid[1].p;
  b.adj = (const int32_t*)adj.p;
  b.run_delta = (const int32_t*)delta.p;
  b.head_bits = (const uint64_t*)bits.p;
  b.run_base = (const int32_t*)base.p;

  ws.alloc((size_t)ws_bytes, "workspace allocation");
  hipStream_t stream = nullptr;
  check_hip(hipStreamCreate(&stream), "stream");
  lbm_solver* s = nullptr;
  check(lbm_solver_create(&p, &b, ws.p, ws_bytes, stream, &s), "solver create");
  if (!sched.empty()) {
    sched_dev.alloc(sched.size() * sizeof(int32_t), "schedule allocation");
    check(lbm_solver_set_odd_schedule(s, sched.data(), (int64_t)sched.size(), (int32_t*)sched_dev.p), "odd schedule");
  }
  check(lbm_solver_init_equilibrium(s, nullptr, nullptr), "init");
  check(lbm_solver_step(s, steps), "step");

  std::vector<double> f((size_t)(19 * N)), tot(4, 0.0);
  f_dev.alloc(f.size() * sizeof(double), "export allocation");
  tot_dev.alloc(4 * sizeof(double), "totals allocation");
  check(lbm_solver_export_pdfs(s, (double*)f_dev.p), "export");
  check(lbm_solver_moments(s, nullptr, nullptr, (double*)tot_dev.p), "moments");
  check_hip(hipStreamSynchronize(stream), "synchronize");
  if (!f.empty()) check_hip(hipMemcpy(f.data(), f_dev.p, f.size() * sizeof(double), hipMemcpyDeviceToHost), "copy");
  check_hip(hipMemcpy(tot.data(), tot_dev.p, 4 * sizeof(double), hipMemcpyDeviceToHost), "copy");
  int64_t t = 0;
  check(lbm_solver_time(s, &t), "time");
  lbm_solver_free(s);
  check_hip(hipStreamDestroy(stream), "stream");

  FILE* fo = std::fopen(argv[16], "wb");
  if (!fo) die("cannot open output", argv[16]);
  bool ok = std::fwrite(&N, sizeof N, 1, fo) == 1;
  ok = ok && std::fwrite(node_voxel.data(), sizeof(int32_t), node_voxel.size(), fo) == node_voxel.size();
  ok = ok && std::fwrite(f.data(), sizeof(double), f.size(), fo) == f.size();
  ok = (std::fclose(fo) == 0) && ok;
  if (!ok) die("cannot write output", argv[16]);
  std::printf("N=%lld runs=%lld t=%lld mass=%.17g jx=%.17g jy=%.17g jz=%.17g\n", (long long)N,
              (long long)runs_used, (long long)t, tot[0], tot[1], tot[2], tot[3]);
  return 0;
}
