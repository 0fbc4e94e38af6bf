/*
 * lbm_sparse.h - C ABI of the sparse-lattice D3Q19 lattice Boltzmann library
 * for AMD Instinct MI355X (gfx950).
 *
 * Method: Wittmann, Zeiser, Hager, Wellein, "Modeling and analyzing
 * performance for highly optimized propagation steps of the lattice Boltzmann
 * method on sparse lattices" (arXiv:1410.0412).
 *
 * Only fluid nodes are stored (Sect. 1). Their order is fixed by an
 * enumeration function: lexicographic sorting with a blocking factor, or a
 * space-filling curve (Sect. 1, Sect. 5.6, Sect. 6). Neighbours are reached
 * through an adjacency list of 18 four-byte indices per node (Sect. 4, Loop
 * Balance). One time step is a fused collide-and-propagate update of
 * eq. (1) (Sect. 2) in one of two propagation patterns (Sect. 4): the
 * two-grid one-step pull algorithm (OS-NT) or the one-grid AA pattern, each
 * with plain indirect addressing or with reduced indirect addressing (RIA,
 * Sect. 4.1), which run-length codes nodes whose access pattern is that of
 * the previous node shifted by one.
 *
 * Conventions
 * - Every function returns 0 (LBM_OK) on success or a negative LBM_E* code;
 *   lbm_last_error() then returns a message (per thread, valid until the next
 *   failing call on that thread). No C++ exception crosses this interface.
 * - Voxel boxes are nx*ny*nz, C order: voxel id = (x*ny + y)*nz + z.
 * - D3Q19 directions q = 0..18: 0 rest; 1 +x, 2 -x, 3 +y, 4 -y, 5 +z, 6 -z;
 *   7 (+1,+1,0), 8 (-1,-1,0), 9 (+1,-1,0), 10 (-1,+1,0), 11 (+1,0,+1),
 *   12 (-1,0,-1), 13 (+1,0,-1), 14 (-1,0,+1), 15 (0,+1,+1), 16 (0,-1,-1),
 *   17 (0,+1,-1), 18 (0,-1,+1). Opposite of odd q is q+1, of even q>0 is q-1.
 * - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *   memory of the current device. The library never allocates device
 *   memory: callers pass every device buffer and keep it alive until the
 *   work queued on it has finished.
 * - Device work is queued asynchronously on the HIP stream given to the
 *   solver; errors of queued kernels surface as LBM_EDEVICE at a later call
 *   that synchronises (moments, export) or checks the launch status.
 * - Handles are not thread-safe; use one handle per thread.
 */
#ifndef LBM_SPARSE_H
#define LBM_SPARSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,  /* invalid argument (null pointer, bad size or flag)   */
  LBM_ERANGE = -2,  /* a size does not fit the index type                  */
  LBM_ENOMEM = -3,  /* host allocation failed                              */
  LBM_EDEVICE = -4, /* HIP runtime error                                   */
  LBM_ESTATE = -5   /* call not valid in the object's current state        */
};

enum { LBM_ORDER_LEX = 0, LBM_ORDER_MORTON = 1, LBM_ORDER_HILBERT = 2, LBM_ORDER_HILBERT_LS = 3 };
enum { LBM_PATTERN_AA = 0, LBM_PATTERN_OSNT = 1 };
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16 = 2 };
enum { LBM_BGK = 0, LBM_TRT = 1 };
/* Neighbour index source of a solver (lbm_params.ria): the adjacency list,
 * the paper's runs (Sect. 4.1) or per-direction runs. */
enum { LBM_INDEX_ADJ = 0, LBM_INDEX_RUNS = 1, LBM_INDEX_DIRECTION_RUNS = 2 };
/* Solver flags. LBM_FLAG_NO_XCD_REMAP: launch the step kernels in plain tile
 * order. By default each XCD takes chunks of consecutive 256-node tiles in
 * turn, so neighbouring tiles share an L2. LBM_FLAG_WIDE_SLOTS: step with
 * 64-bit slot offsets whatever the grid size; without it they are 64-bit
 * only for grids of more than 2^31 - 1 elements. Both forms compute the same
 * result bit for bit; the flag exercises the wide form on small lattices. */
enum { LBM_FLAG_NO_XCD_REMAP = 1, LBM_FLAG_WIDE_SLOTS = 2 };

/* Message of the last failing call on this thread ("" if none). */
const char* lbm_last_error(void);

/* ====================================================================== */
/* Host lattice: enumeration, adjacency list, RIA runs, wave tables        */
/* ====================================================================== */

typedef struct lbm_lattice lbm_lattice;

/*
 * Build the sparse lattice of a voxel mask (host, synchronous).
 *
 * solid          host, nx*ny*nz bytes, C order; nonzero marks a solid voxel.
 * periodic_mask  bit 0/1/2: x/y/z axis periodic. On a non-periodic axis the
 *                outside of the box counts as solid (halfway bounce-back).
 * order          LBM_ORDER_LEX: lexicographic sorting (Sect. 5.6), x slowest
 *                and z fastest, visiting block x block x block tiles in that
 *                order and voxels inside a tile in that order; block = 0 (or
 *                >= the largest extent, or 1) means no blocking.
 *                LBM_ORDER_MORTON: Morton space-filling curve (bits of x, y, z
 *                interleaved, x most significant per triple); block ignored.
 *                LBM_ORDER_HILBERT: Hilbert curve on the bounding 2^b cube
 *                (the space-filling curve of Sect. 5.6); block ignored.
 *                LBM_ORDER_HILBERT_LS: two-stage renumbering of Sect. 6.1:
 *                the Hilbert order is cut into `block` (>= 1) contiguous
 *                chunks of ceil(N/block) nodes, each re-enumerated by plain
 *                lexicographic order.
 *
 * Node n is the n-th fluid voxel in that order. For q = 1..18 the adjacency
 * entry of node n is the node at the upstream site x_n - c_q (pull scheme,
 * Sect. 4), or -1 if that site is solid or outside the box. Runs (Sect. 4.1):
 * node n > 0 continues the run of node n-1 iff for every q its entry equals
 * the entry of n-1 plus one, or both are -1; runs are maximal.
 *
 * Errors: LBM_EINVAL for null pointers or non-positive extents or a negative
 * block; LBM_ERANGE if nx*ny*nz or the fluid-node count exceeds 2^31-1 or an
 * extent exceeds 2^21 (Morton); LBM_ENOMEM. On success *out owns all tables
 * until lbm_lattice_free.
 */
int lbm_lattice_build(const uint8_t* solid, int32_t nx, int32_t ny, int32_t nz,
                      uint32_t periodic_mask, int32_t order, int32_t block,
                      lbm_lattice** out);

/* Table sizes: N fluid nodes, R runs, W = ceil(N/64) wavefront tiles. */
int lbm_lattice_sizes(const lbm_lattice* lat, int64_t* n_fluid, int64_t* n_runs,
                      int64_t* n_waves);

/* node_voxel: host int32[N]; voxel id of node n. */
int lbm_lattice_copy_nodes(const lbm_lattice* lat, int32_t* node_voxel);

/* adj: host int32[18*ld], ld >= N; entry of direction q (1..18) for node n at
 * adj[(q-1)*ld + n]. Columns N..ld-1 are filled with -1. The lattice stores
 * no adjacency list (72 B per node); this call computes it from the
 * voxel-to-node map the lattice keeps (4 B per voxel). */
int lbm_lattice_copy_adjacency(const lbm_lattice* lat, int32_t* adj, int64_t ld);

/* run_start: host int32[R+1]; first node of each run, then N (the block
 * vector of Sect. 4.1 stored as prefix sums of the run lengths). */
int lbm_lattice_copy_runs(const lbm_lattice* lat, int32_t* run_start);

/*
 * Per-wavefront RIA encoding (64-node tiles; one GPU lane per node):
 * run_delta  host int32[18*ldr], ldr >= R: for run r with head h,
 *            run_delta[(q-1)*ldr + r] = adj_q(h) - h, or INT32_MIN if
 *            adj_q(h) = -1. Inside run r, adj_q(n) = n + run_delta.
 *            Columns R..ldr-1 are filled with INT32_MIN.
 * head_bits  host uint64[W]; bit l of word w set iff node 64w+l heads a run.
 * run_base   host int32[W]; (number of run heads below node 64w) - 1.
 * Node 64w+l lies in run run_base[w] + popcount(head_bits[w] & bits 0..l).
 */
int lbm_lattice_copy_wave_tables(const lbm_lattice* lat, int32_t* run_delta, int64_t ldr,
                                 uint64_t* head_bits, int32_t* run_base);

/*
 * Per-direction runs (a GPU encoding of the idea of Sect. 4.1, not part of
 * the paper): the run rule applied to each direction q on its own, so a run
 * of direction q only ends where the entries of q stop shifting by one (the
 * paper's runs end where any direction does). Runs of direction q are
 * numbered after those of directions 1..q-1; RD is their total.
 * LBM_ERANGE if RD exceeds 2^31-1.
 */
int lbm_lattice_direction_runs(const lbm_lattice* lat, int64_t* n_dir_runs);

/*
 * Per-direction wave tables (any pointer may be NULL, then skipped):
 * dir_delta  host int32[RD]: adj_q(h) - h for the run of direction q whose
 *            first node is h, or INT32_MIN if adj_q(h) = -1.
 * dir_bits   host uint64[18*W]; word 18w + q-1 has bit l set iff node 64w+l
 *            starts a run of direction q.
 * dir_base   host int32[18*W]; entry 18w + q-1 = (index of the first run of
 *            direction q) + (direction-q run starts below node 64w) - 1.
 * For node n = 64w+l: k = 18w + q-1, r = dir_base[k] +
 * popcount(dir_bits[k] & bits 0..l), and adj_q(n) = n + dir_delta[r].
 * LBM_ERANGE if RD exceeds 2^31-1.
 */
int lbm_lattice_copy_direction_tables(const lbm_lattice* lat, int32_t* dir_delta,
                                      uint64_t* dir_bits, int32_t* dir_base);

/*
 * Workgroup order for the AA odd step on large lattices (an extension
 * beyond the paper, for the cache hierarchy of a multi-die GPU). The step
 * kernels run one workgroup per block of 256 consecutive nodes, and the
 * device deals workgroup b to die (XCD) b mod 8. In the default order all 8
 * XCDs sweep the node list together, so a block and its x-neighbours one
 * x-plane away meet one plane's sweep apart, mostly on different XCDs; once a
 * plane's traffic outgrows the caches, the lines they share are fetched and
 * written back twice. The band schedule sweeps y-bands of band_rows rows one
 * after the other, and inside a band x-plane after x-plane; XCD k takes the
 * blocks whose first node lies in rows [k, k + 1) * band_rows / 8 of the
 * band, so a block's x-neighbours follow on the same XCD soon after.
 * sched: host int32[*len] or NULL. With NULL, *len receives the length the
 * schedule needs (a multiple of 8). Otherwise *len must be at least that
 * length; on return sched[8 j + k] is the j-th block of XCD k, or -1 (no
 * work), and *len the length written. Only for LS order without blocking
 * (x slowest, z fastest). Errors: LBM_EINVAL (null lattice or len, another
 * order, band_rows not a positive multiple of 8, *len too small).
 */
int lbm_lattice_band_schedule(const lbm_lattice* lat, int32_t band_rows, int32_t* sched, int64_t* len);

void lbm_lattice_free(lbm_lattice* lat);

/* ====================================================================== */
/* Device solver                                                           */
/* ====================================================================== */

typedef struct lbm_params {
  double tau;        /* BGK relaxation time, > 1/2                           */
  double force[3];   /* constant body-force density F                       */
  double rho0;       /* reference density of deviation storage (> 0)        */
  int32_t pattern;   /* LBM_PATTERN_AA or LBM_PATTERN_OSNT                   */
  int32_t ria;       /* LBM_INDEX_ADJ: adjacency list; LBM_INDEX_RUNS: RIA
                        wave tables; LBM_INDEX_DIRECTION_RUNS: per-direction
                        RIA tables                                           */
  int32_t precision; /* LBM_F64: FP64 storage and arithmetic. LBM_F32: the
                        grid stores d_q = f_q - w_q*rho0 in FP32. LBM_F16: it
                        stores d_q * 2^f16_scale_log2 / w_q in FP16. Both
                        deviation formats collide in FP32; moments, totals and
                        export/import are FP64.                              */
  int32_t flags;     /* LBM_FLAG_NO_XCD_REMAP | LBM_FLAG_WIDE_SLOTS, or 0   */
  int64_t n_fluid;   /* N                                                    */
  int64_t n_runs;    /* R (LBM_INDEX_RUNS) or RD (LBM_INDEX_DIRECTION_RUNS) */
  int64_t ldf;       /* node slots of the grid: >= N, a multiple of 64,
                        <= 2^31. Grid layout (tile-major SoA): direction q
                        of node n = 64t + l is element (19t + q)*64 + l; a
                        grid holds 19*ldf elements. Grids of up to 2^31 - 1
                        elements (N up to 113 M) step with 32-bit element
                        offsets, larger ones with 64-bit offsets: one FP64
                        AA grid can fill the whole of a 288 GB device.     */
  int64_t lda;       /* adjacency row stride (>= N, <= 2^31), adjacency only */
  int64_t ldr;       /* run_delta row stride (>= R, <= 2^31), LBM_INDEX_RUNS
                        only                                                 */
  int32_t f16_scale_log2; /* FP16 storage scale exponent s, in [-24, 24]     */
  int32_t collision; /* LBM_BGK, or LBM_TRT (two relaxation times, Sect. 2):
                        f*_q = f_q - w+ (f+_q - feq+_q) - w- (f-_q - feq-_q)
                        + S_q with w+ = 1/tau and w- fixed by trt_magic      */
  double trt_magic;  /* TRT: Lambda = (1/w+ - 1/2)(1/w- - 1/2) > 0           */
} lbm_params;

typedef struct lbm_buffers {
  void* pdf[2];               /* device PDF grids, 19*ldf elements of the
                                 storage type (double, float or IEEE half)
                                 each, tile-major (see ldf); pdf[1] only for
                                 OS-NT                                       */
  const int32_t* adj;         /* device [18][lda] (LBM_INDEX_ADJ)            */
  const int32_t* run_delta;   /* device [18][ldr] (LBM_INDEX_RUNS), or
                                 dir_delta [RD] (LBM_INDEX_DIRECTION_RUNS)   */
  const uint64_t* head_bits;  /* device [W], or dir_bits [W][18]             */
  const int32_t* run_base;    /* device [W], or dir_base [W][18]             */
  const double* solid_frac;   /* device [N] partial-bounce-back solid
                                 fraction ns in [0, 1] per node, or NULL.
                                 With it every step applies
                                 post_q = (1 - ns) f*_q + ns f_qbar after the
                                 BGK collision (AA pattern, FP64, BGK only). */
} lbm_buffers;

typedef struct lbm_solver lbm_solver;

/* Workspace bytes the solver needs (device scratch for reductions). */
int lbm_solver_workspace_bytes(const lbm_params* p, int64_t* bytes);

/*
 * Device bytes a caller allocates for a solver with parameters p (host,
 * touches no device): *pdf_bytes_per_grid = 19 * ldf * (8, 4 or 2 bytes per
 * stored PDF of LBM_F64, LBM_F32, LBM_F16), the size of one PDF grid
 * (Sect. 4: 19 PDFs per fluid node; one grid for the AA pattern, two for
 * OS-NT), and *workspace_bytes as lbm_solver_workspace_bytes. Only
 * precision, n_fluid and ldf are read; ldf = 0 asks for the smallest valid
 * stride, N rounded up to a multiple of 64 (at least 64). The index tables
 * are sized by the lattice (lbm_lattice_sizes, lbm_lattice_direction_runs).
 * Errors: LBM_EINVAL (null pointer, unknown precision, n_fluid < 0, ldf < N
 * or not a multiple of 64), LBM_ERANGE (N above 2^31 - 65, ldf above 2^31).
 */
int lbm_required_bytes(const lbm_params* p, int64_t* pdf_bytes_per_grid, int64_t* workspace_bytes);

/*
 * Create a solver over caller-owned device buffers (borrowed, not copied).
 * workspace: device, at least lbm_solver_workspace_bytes. hip_stream: the
 * hipStream_t all work is queued on (NULL: the default stream). The solver
 * starts at t = 0 with undefined PDFs; call an init or import first.
 * Errors: LBM_EINVAL (tau <= 1/2, bad flags, missing buffers, ldf < N or not
 * a multiple of 64, lda < N, ldr < R, per-direction tables with fewer than 18
 * runs), LBM_ERANGE (N above 2^31 - 65, ldf, lda or ldr above 2^31, or
 * more than 2^31 - 1 per-direction runs), LBM_ENOMEM.
 * Creation touches no device; the device limits used by the launches are
 * read at the first step.
 */
int lbm_solver_create(const lbm_params* p, const lbm_buffers* b, void* workspace,
                      int64_t workspace_bytes, void* hip_stream, lbm_solver** out);

/* Set the stream later work is queued on. */
int lbm_solver_set_stream(lbm_solver* s, void* hip_stream);

/*
 * Launch the AA odd step's workgroups in the order sched (host int32[len],
 * len a positive multiple of 8: entry b names the 256-node block that
 * workgroup b processes, -1 an empty slot; every block of the lattice must
 * appear exactly once), as lbm_lattice_band_schedule makes it. The library
 * checks the schedule on the host, copies it into sched_device (a
 * caller-owned device int32[len] that must outlive the solver's use of it;
 * the call synchronises the stream) and launches the odd step with len
 * workgroups from then on. sched = NULL restores the default order. The
 * even step, OS-NT and the partial-bounce-back and adjoint steps keep the
 * default order. A step's result does not depend on the order.
 * Errors: LBM_EINVAL (null solver or sched_device, a bad len, an entry
 * outside [-1, number of blocks), a block missing or twice), LBM_ESTATE
 * (OS-NT pattern), LBM_EDEVICE (the copy failed).
 */
int lbm_solver_set_odd_schedule(lbm_solver* s, const int32_t* sched, int64_t len, int32_t* sched_device);

/*
 * f(0) = feq(rho, u) on every node and t = 0 (one kernel).
 * rho: device double[N] or NULL (rho0 everywhere); u: device double[3*N]
 * (component-major: u[a*N + n]) or NULL (zero velocity).
 */
int lbm_solver_init_equilibrium(lbm_solver* s, const double* rho, const double* u);

/*
 * Advance n_steps time steps (one kernel launch per step, asynchronous).
 * AA: even t runs the direct step, odd t the indirect step (Sect. 4);
 * OS-NT: pull step into the other grid, then the grids swap. Workgroups take
 * tiles in XCD-aware chunks (unless LBM_FLAG_NO_XCD_REMAP), and the
 * streaming kernels reserve LDS they do not use, to cap their occupancy.
 */
int lbm_solver_step(lbm_solver* s, int64_t n_steps);

/* Current time step t. */
int lbm_solver_time(const lbm_solver* s, int64_t* t);

/*
 * Macroscopic fields of the pre-collision PDFs f(t): rho[n] and
 * u[a*N + n] = j_a / rho (device double, either may be NULL), and totals
 * (device double[4]: mass, jx, jy, jz summed over all nodes in a fixed
 * order; may be NULL). Synchronises the stream. The totals are always
 * formed (in the workspace) and checked on the host: LBM_ERANGE if one is
 * NaN or infinite, i.e. some PDF is (the outputs are still written).
 */
int lbm_solver_moments(lbm_solver* s, double* rho, double* u, double* totals);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same as
 * lbm_solver_moments, but the partial sums go to a scratch array of
 * (1024 * 4 + 4) doubles (32,800 bytes) that the library keeps in static
 * device memory, one copy per device, instead of the solver's workspace.
 * Results are bitwise those of lbm_solver_moments. The call allocates no
 * device memory (the first call on a device looks up the array's address).
 * Every call on a device shares that device's array: calls that overlap in
 * time on one device (other threads, other streams) race and must be
 * serialised by the caller. Nothing in it needs clearing between calls: a
 * call writes every partial sum it reads. The partial sums need at most the array's size
 * for any lattice; LBM_ERANGE otherwise. Synchronises the stream.
 */
int lbm_solver_moments_static(lbm_solver* s, double* rho, double* u, double* totals);

/* f(t) in natural order: device double[19*N], f[q*N + n]. Synchronises. */
int lbm_solver_export_pdfs(lbm_solver* s, double* f);

/* Set the state to f (device double[19*N], natural order) at time t >= 0. */
int lbm_solver_import_pdfs(lbm_solver* s, const double* f, int64_t t);

/* Declare that the AA grid currently holds the state of time t (layout by
 * parity), e.g. after the caller copied a checkpoint into pdf[0].
 * LBM_ESTATE for OS-NT. */
int lbm_solver_set_time(lbm_solver* s, int64_t t);

/* out (device double[1]) = sum_n weight[n] * j_axis(n, t) of f(t), FP64,
 * in a fixed summation order. weight: device double[N]. Synchronises. */
int lbm_solver_weighted_momentum(lbm_solver* s, const double* weight, int32_t axis, double* out);

void lbm_solver_free(lbm_solver* s);

/* ====================================================================== */
/* Adjoint of the AA step (AA pattern, FP64, BGK, optional partial         */
/* bounce-back). Not part of the paper: the differentiation extension.     */
/* ====================================================================== */

/*
 * lam (device double[19*ldf], the tile-major AA slot layout of time t) = dJ/df(t) for
 * J = sum_n weight[n] * j_axis(n, t): lam at the slot of f_q(n) is
 * weight[n] * c_q,axis. Asynchronous.
 */
int lbm_adjoint_seed_momentum(lbm_solver* s, const double* weight, int32_t axis, int64_t t,
                              double* lam);

/*
 * One AA step t -> t+1 that also writes the PDFs f(t) it reads into save
 * (device double[19*ldf], not the solver's grid): afterwards save holds, at
 * every slot of a fluid node, what the AA grid held before the step, which is
 * the forward state lbm_adjoint_step needs for step t. Slots of the padding
 * nodes N..ldf-1 are not written. The step itself is that of
 * lbm_solver_step(s, 1): with partial bounce-back if the solver has a
 * solid-fraction buffer, else the plain step (bitwise). It costs 8 B per PDF
 * written, against a read and a write per PDF for a copy of the grid.
 * Asynchronous. LBM_EINVAL for a null pointer or save equal to the grid;
 * LBM_ESTATE unless AA, FP64 and BGK.
 */
int lbm_solver_step_save(lbm_solver* s, double* save);

/*
 * Backward through the step t -> t+1. fwd: device double[19*ldf], the AA grid
 * holding f(t) (as the solver held it before stepping from t). lam: on entry
 * dJ/df(t+1) in the layout of time t+1, on exit dJ/df(t) in the layout of
 * time t (in place). grad (device double[N] or NULL): dJ/dns(n) accumulates
 * sum_q mu_q (f_qbar - f*_q), mu_q = dJ/dpost_q. Asynchronous. LBM_ESTATE
 * unless AA, FP64 and BGK.
 */
int lbm_adjoint_step(lbm_solver* s, const double* fwd, int64_t t, double* lam, double* grad);

/* ====================================================================== */
/* Bandwidth micro-benchmarks (Sect. 5.2, Table 3, GPU analogues)          */
/* ====================================================================== */

/*
 * kind 0 "copy": dst[i] = src[i] for n doubles (STREAM copy).
 * kind 1 "CNT-19A": 19 streams of n doubles, stride ld, copied src -> dst
 *        (the traffic pattern of the OS-NT step).
 * kind 2 "U-19A": 19 streams of n doubles, stride ld, updated in place in dst
 *        (the traffic pattern of the AA even step); src unused.
 * kind 3 "U-1A": one stream of n doubles updated in place in dst; src unused.
 * kind 4 "CNT-1A": copy of one stream of n doubles (same as kind 0).
 * kind 5 "U-19T": the U-19A update in the tile-major layout of the PDF grid
 *        (19 rows of 64 doubles per 64-node tile, in place in dst; needs
 *        ld >= n rounded up to 64, dst of 19*ld doubles); src unused.
 * kind 6 "CNT-19T": the CNT-19A copy in the tile-major layout, src -> dst
 *        (both 19*ld doubles, ld >= n rounded up to 64).
 * kind 7 "U-19T-L": U-19T launched as the FP64 AA even step is (XCD-aware
 *        chunks of 64 workgroups, 2 workgroups per CU).
 * kind 8 "CNT-19T-L": CNT-19T in the same launch (the fastest of chunks of
 *        0, 16 or 64 workgroups with 2 or 5 workgroups per CU, or no cap).
 * Asynchronous on hip_stream.
 */
int lbm_bench_stream(int32_t kind, const double* src, double* dst, int64_t n, int64_t ld,
                     void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_SPARSE_H */
