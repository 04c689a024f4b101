/*
 * tb.h -- C ABI of the MI355X tensor butterfly library (libtb.so).
 *
 * The library builds and applies the tensor butterfly factorisation of a
 * discretised d-dimensional oscillatory integral operator K with n^d target
 * and n^d source points (Kielstra, Shi, Luo, Qian, Liu, "A Linear-complexity
 * Tensor Butterfly Algorithm for Compressing High-dimensional Oscillatory
 * Integral Operators", arXiv 2411.03029):
 *
 *   tb_construct      Algorithm 1 (construction) on the GPU: FP64 kernel
 *                     entries at proxy indices, column interpolative
 *                     decompositions (section 2.1) by FP64 Householder QR,
 *                     nested over levels (section 3.2), and the middle-level
 *                     cores K(tbar, sbar).
 *   tb_apply          Algorithm 2 (contraction): u = K_BF f.
 *   tb_apply_adjoint  the conjugate-transposed contraction: v = K_BF^H g.
 *
 * Conventions shared by every call
 * --------------------------------
 * Status:    every call returns a tb_status (TB_OK = 0) and never aborts;
 *            tb_last_error() returns a thread-local message for the last
 *            failure on the calling thread.
 * Arrays:    f, u, g, v are caller-owned DEVICE pointers, contiguous, layout
 *            (nrhs, n, ..., n) row-major (mode d fastest), complex values
 *            interleaved (re, im).  Element type by tb_dtype below.  Input
 *            and output must not overlap.
 * Streams:   work is enqueued on the caller's HIP stream (hipStream_t passed
 *            as void*, NULL = default stream) and the calls return without
 *            synchronising, except where a call says otherwise.  A plan owns
 *            its workspace: one stream at a time per plan.
 * Ownership: a plan owns all device memory for factors, cores and
 *            workspace; tb_destroy frees it.
 * Indexing:  target multi-index i and source multi-index j in [0, n)^d.
 *            Fourier (d = 2, 3): K = exp(-2 pi i x.k), x = i/n, k = j - n/2
 *              (section 4.3, phase reduced exactly in integers).
 *            Helmholtz (section 4.1): K = exp(+i omega rho)/rho, rho = |x - y|;
 *              d = 3: x = i/n, y = j/n + (2, 0, 0) (two unit cubes, centres
 *              2 apart along x1); d = 2: x = (i/n, 0), y = (j/n, 1) (two
 *              parallel facing unit plates, 1 apart).
 *            Radon (section 4.2), x = i/n, k = j - n/2, K = exp(2 pi i phi):
 *              d = 2: phi = x.k + sqrt(c1^2 k1^2 + c2^2 k2^2),
 *                c1 = (a + b sin 2pi x1 sin 2pi x2)/den,
 *                c2 = (a + b cos 2pi x1 cos 2pi x2)/den, (a, b, den) = (2, 1, 3)
 *                unless tb_options sets them (the paper's are (2, 1, 16));
 *              d = 3: phi = x.k + c |k|,
 *                c = (a + b sin 2pi x1 sin 2pi x2 sin 2pi x3)/den,
 *                (a, b, den) = (3, 1, 100) unless set.
 *            Non-uniform DFT, type 2 (section 4.3, d = 2, 3): K = exp(2 pi i x.y),
 *              y = j/n, x_k = X[k][i_k] from tb_options.nudft_x.
 *            Uniform DFT (section 4.3, d = 2 .. 6): K = exp(2 pi i br(i).br(j)/n),
 *              the bit-reversal ordering of every mode; phase exact in integers.
 *            Applies with d > 3 run FP64 or FP32 with stored cores, on kernels
 *            generic in the number of modes (no autotuning, no on-the-fly or
 *            compressed cores).
 */
#ifndef TB_H
#define TB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TB_OK = 0,
  TB_ERR_INVALID_ARG = 1,  /* bad argument; nothing was launched            */
  TB_ERR_UNSUPPORTED = 2,  /* valid request this build does not implement   */
  TB_ERR_OOM = 3,          /* device allocation failed or exceeded the cap   */
  TB_ERR_HIP = 4,          /* a HIP runtime call failed (message attached)   */
  TB_ERR_NUMERIC = 5,      /* an ID rank exceeded the allowed maximum        */
  TB_ERR_IO = 6            /* plan file missing, truncated or corrupted      */
} tb_status;

typedef enum {
  TB_KERNEL_FOURIER = 0,
  TB_KERNEL_HELMHOLTZ = 1,
  TB_KERNEL_RADON = 2,
  TB_KERNEL_NUDFT = 3,  /* type-2 non-uniform DFT, section 4.3: K = exp(2 pi i x.y),
                           y = j/n, x_k = X[k][i_k] from tb_options.nudft_x */
  TB_KERNEL_DFT = 4     /* uniform DFT of section 4.3, d = 2 .. 6: K = exp(2 pi i x.y)
                           with x = br(i), y = br(j)/n per mode, br reversing the
                           log2(n) bits (the bit-reversal ordering of each
                           dimension); n a power of two */
} tb_kernel;

/* Element type of the apply.  TB_C128: complex128 arrays, FP64 factors,
 * cores and accumulation.  TB_C64: complex64 arrays, FP32 everything.
 * TB_CBF16: complex64 arrays, BF16 cores, FP32 factors and accumulation.
 * TB_C64_OTF: complex64 arrays, FP32 factors and accumulation, the cores
 * K(tbar, sbar) evaluated inside the core contraction from the skeleton
 * indices (section 2: any entry in O(1)) instead of read from memory: phase
 * formed and reduced to a fraction of a turn in FP64, sine and cosine in
 * FP32; available for every plan, stored cores or not.
 * TB_CQ16: complex64 arrays, FP32 factors and accumulation, cores stored
 * compressed as block-scaled 16-bit fixed point (a fixed-rate core codec in
 * the spirit of the paper's ZFP-compressed cores, section 3.2 and Algorithm 2
 * step 2): one FP32 scale
 * per core column (its largest real or imaginary magnitude / 32767) and two
 * int16 per entry, 4 bytes per complex entry; decoded inside the core
 * contraction.  Per entry the error is at most half a step, 2^-16 of the
 * column's largest part. */
typedef enum { TB_C128 = 0, TB_C64 = 1, TB_CBF16 = 2, TB_C64_OTF = 3, TB_CQ16 = 4 } tb_dtype;

#define TB_STORE_C128 (1u << TB_C128)
#define TB_STORE_C64 (1u << TB_C64)
#define TB_STORE_CBF16 (1u << TB_CBF16)
/* store_mask == TB_STORE_OTF keeps no cores: only TB_C64_OTF applies run. */
#define TB_STORE_OTF (1u << TB_C64_OTF)
#define TB_STORE_CQ16 (1u << TB_CQ16)

typedef struct tb_plan_s* tb_plan;

/* Construction options.  A zero-initialised struct (or NULL) gives the
 * defaults listed per field. */
typedef struct {
  int leaf_size;        /* C_b, indices per leaf per mode; 0 -> 8            */
  int lt_override;      /* 0 -> target middle level ceil(L/2); v > 0 sets
                           it to v - 1 (source middle level = L - that)     */
  int proxy_pair;       /* samples of the paired mode per ID column; 0 -> 2;
                           < 0 -> every index of the node                  */
  int proxy_other;      /* samples of every other mode; 0 -> 4*leaf (d = 2)
                           or 4 (d = 3); < 0 -> every index of the node     */
  double id_tol_scale;  /* ID tolerance = id_tol_scale * tol; 0 -> 0.3      */
  unsigned store_mask;  /* core precisions kept (TB_STORE_*); 0 -> C64;
                           TB_STORE_OTF alone keeps none                   */
  int max_rank;         /* > 0: an ID rank above it fails with
                           TB_ERR_NUMERIC; 0 -> no limit                   */
  size_t max_device_bytes; /* > 0: cap on the plan's device memory; a plan
                              that needs more fails with TB_ERR_OOM         */
  int radon_custom;     /* 1: use radon_a/b/den below; 0 -> a=2, b=1, den=3
                           (d = 2) or the section 4.2 a=3, b=1, den=100
                           (d = 3)                                         */
  double radon_a, radon_b, radon_den;
  const double* nudft_x; /* TB_KERNEL_NUDFT (required): host array of d * n
                            target coordinates, mode k at [k n, (k + 1) n),
                            each in [0, n - 1] and non-decreasing within a
                            mode (index blocks are then coordinate
                            intervals); copied into the plan              */
} tb_options;

/* Summary of a plan (tb_plan_info). */
typedef struct {
  int kind, d, leaf;
  long long n;
  int L, Lt, Ls;              /* levels; target / source middle levels      */
  int r_min, r_max;           /* over all IDs                               */
  long long n_ids;            /* number of IDs (source + target)            */
  long long n_pairs;          /* middle-level (t, s) pairs                  */
  long long factor_entries;   /* true-rank V, W, U, P entries               */
  long long core_entries;     /* true-rank core entries, sum of R_T * R_S    */
  long long core_rows;        /* sum over pairs of R_T                      */
  long long core_cols;        /* sum over pairs of R_S                      */
  long long apply_cmacs;      /* complex multiply-adds of one apply per RHS,
                                 counted from the true ranks                */
  double omega, tol, eps_id;
  unsigned store_mask;
  size_t device_bytes;        /* factor + core memory held by the plan      */
  double construct_ms;        /* wall time of tb_construct (0 after load)   */
  long long stage_cmacs[5];   /* apply_cmacs split by forward stage: source
                                 leaf, source transfers (all levels), core,
                                 target transfers, target leaf; the adjoint
                                 stage mirroring each has the same count    */
  long long stage_io_entries[5]; /* per RHS, the same split: entries of the
                                 tensors the stage family reads and writes
                                 (true ranks, each tensor once; the leaves
                                 include the n^d array, the core family F
                                 and G but not the cores)                   */
} tb_plan_info_t;

/* Build the factorisation on the GPU (Algorithm 1).
 *   kind, d:  operator, d in {2, 3} for every kind; also 4 .. 6 for
 *             TB_KERNEL_DFT.  Fourier: K =
 *             exp(-2 pi i x.k), x = i/n, k = j - n/2 (section 4.3).
 *             Helmholtz: exp(+i omega rho)/rho; d = 3 two unit cubes with
 *             centres 2 apart along x1, d = 2 two parallel facing unit
 *             plates 1 apart (section 4.1).  Radon: exp(2 pi i phi), x =
 *             i/n, k = j - n/2; d = 2 phi = x.k + sqrt(c1^2 k1^2 + c2^2
 *             k2^2), d = 3 phi = x.k + c |k| (section 4.2 equations).
 *   n:        points per direction; n = leaf * 2^L with L >= 0.
 *   omega:    Helmholtz wavenumber (> 0); ignored for Fourier and Radon.
 *   tol:      requested relative accuracy in (0, 1); every ID runs at
 *             id_tol_scale * tol (section 2.1 Frobenius criterion).
 *   opt:      options or NULL.  hip_stream: stream for the GPU work.
 *   out:      receives the plan.
 * Synchronises with the device once per tree level (ranks are read back to
 * size the next level).  Errors: TB_ERR_INVALID_ARG for a bad d/n/tol/omega,
 * TB_ERR_UNSUPPORTED for a (kind, d) pair not built, TB_ERR_NUMERIC if an ID
 * exceeds opt->max_rank, TB_ERR_OOM, TB_ERR_HIP. */
tb_status tb_construct(tb_kernel kind, int d, long long n, double omega,
                       double tol, const tb_options* opt, void* hip_stream,
                       tb_plan* out);

/* u = K_BF f (Algorithm 2): f and u hold nrhs >= 1 right-hand sides.
 * io selects the element type (the plan must hold cores of that precision,
 * see store_mask). */
tb_status tb_apply(tb_plan p, const void* f, void* u, long long nrhs,
                   tb_dtype io, void* hip_stream);

/* v = K_BF^H g: the butterfly with every factor conjugate-transposed and
 * the order reversed (not in the paper; the adjoint of Algorithm 2). */
tb_status tb_apply_adjoint(tb_plan p, const void* g, void* v, long long nrhs,
                           tb_dtype io, void* hip_stream);

/* Allocation-free apply, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): u = K_BF f (adjoint == 0) or v = K_BF^H g (adjoint != 0),
 * with the same kernels, launch shapes and results as tb_apply /
 * tb_apply_adjoint.  The intermediates live in a static device array of
 * TB_NOALLOC_SCRATCH_BYTES owned by the library (one per GPU, held until the
 * process ends) instead of the plan's workspace; the call makes no
 * hipMalloc, hipFree or event creation (per-stage timing is not recorded).
 * Arrays and streams as for tb_apply.  Every call on one GPU shares that
 * array and leaves its contents behind: calls that overlap on one GPU (other
 * streams, other threads, other plans) race, and must be serialised by the
 * caller.  A request whose intermediates need more than the array holds
 * fails with TB_ERR_OOM before any launch (the message gives the size);
 * other errors as tb_apply. */
#define TB_NOALLOC_SCRATCH_BYTES (256ull << 20)
tb_status tb_apply_noalloc(tb_plan p, const void* in, void* out, long long nrhs,
                           tb_dtype io, int adjoint, void* hip_stream);

/* Several operators in one submission: plan i maps in[i] -> out[i] with
 * nrhs[i] right-hand sides (forward, or adjoint if adjoint != 0), all of
 * element type io.  The plans' kernel sequences are the parallel branches of
 * one HIP graph, captured on the first call for a given (plans, pointers,
 * nrhs, direction, io) and replayed as a single graph launch on hip_stream by
 * later calls with the same arguments.  Up to 32 graphs are cached (oldest
 * dropped first); a graph is also dropped by tb_batched_reset, by the
 * destruction of one of its plans and when a plan's workspace has to grow.
 * Plans must be distinct; each plan's workspace is shared with its tb_apply
 * calls, so calls on one plan from different streams race.  Arrays as for
 * tb_apply.  A capturing call synchronises the device (workspaces are
 * allocated before capture); the legacy null stream is not captured (a
 * private stream is) but the replay runs on it. */
tb_status tb_apply_batched(int nplans, const tb_plan* plans, const void* const* in,
                           void* const* out, const long long* nrhs, int adjoint,
                           tb_dtype io, void* hip_stream);

/* Drop every cached batched graph (call before freeing captured arrays). */
tb_status tb_batched_reset(void);

/* Autotuner for the launch shapes of every kernel of tb_apply and
 * tb_apply_adjoint on p for nrhs right-hand sides of element type io.
 * Per launch it times the candidates (transfer stages: right-hand sides per
 * workgroup 1/2/4/8, outputs per thread 1/8, sliced or whole blocks; core:
 * vector kernels for 1 or 4 right-hand sides per pass, matrix cores for FP32
 * and BF16) with HIP events on zero-filled scratch buffers it allocates and
 * frees, and keeps the fastest; later applies with exactly this (nrhs, io),
 * batched ones included, use it (other shapes keep the built-in heuristic).
 * cache_path (nullable): a text file of earlier results, one line per
 * (plan signature, io, nrhs); a hit skips the trials, a miss appends the new
 * line.  The signature hashes the construction inputs and every rank, so a
 * line only matches a plan with identical launch shapes.  *trials (nullable)
 * receives the number of configurations timed (0 on a cache hit).
 * Synchronises hip_stream; drops cached batched graphs of p. */
tb_status tb_plan_autotune(tb_plan p, long long nrhs, tb_dtype io, const char* cache_path,
                           void* hip_stream, int* trials);

/* Launch configuration of one kernel of the apply sequence; 0 in a field
 * keeps the built-in heuristic for it. */
typedef struct {
  int outputs_per_thread; /* transfer stages: 1 or 8 */
  int rhs_tile;           /* transfer stages: right-hand sides per workgroup, 1/2/4/8 */
  int whole_blocks;       /* transfer stages: 1 = one workgroup per block (no slices) */
  int core_kernel;        /* core: 1 = vector, 1 RHS per pass; 2 = vector, 4; 3 = FP32 matrix
                             cores (stored or, for TB_C64_OTF, on-the-fly entries); 4 = BF16
                             matrix cores (BF16 applies; right-hand sides split
                             into bf16 hi + lo); 5, 6, 7 = BF16 matrix cores, second form, with
                             256 x 32, 128 x 64, 128 x 32 (rows x right-hand sides) per
                             workgroup; 8, 9 = adjoint vector
                             kernel with 16-lane column groups, 1 or 4 RHS per pass
                             (adjoint launches only) */
  int fanin_in_turn;      /* fan-in stages: 1 = children in turn, first mode in registers;
                             2 = children in turn, first mode first, the coarse slice summed
                             in LDS (8 outputs per thread) */
  int transfer_mfma;      /* transfer levels (not the leaves), FP32 / BF16 applies: 1 = mode
                             products on the matrix cores, one block per workgroup; 2 = d = 3
                             levels on 4 x 4 matrix-core blocks, four right-hand sides per
                             workgroup (fine ranks up to 8, coarse blocks up to 16 per mode):
                             fan-ins take the children in turn and accumulate the coarse
                             block in registers, a group of rows at a time; fan-outs take one
                             fine block per workgroup in two halves of its first mode; also
                             the fan-in leaves (target leaf, source leaf of the adjoint) with
                             leaf size 8 */
  int rhs_per_thread;     /* fan-out / fan-in kernels: 1 or 4 right-hand sides per thread
                             (4 needs a right-hand-side tile of 4 or 8) */
  int flat_stage;         /* transfer stages and leaves: 1 = flat staging (FP32 applies), one
                             right-hand side per workgroup: the block (fan-out: the coarse
                             block; fan-in: all children's blocks) and every matrix loaded
                             into LDS in one pass, then all mode products from LDS; slices
                             for about 1024 workgroups, or whole blocks with whole_blocks = 1;
                             2 = register fibers (FP32 or FP64), one right-hand side per
                             workgroup: each mode product loads fibers of its contracted mode
                             into registers and reads the matrices from LDS; contracted
                             extents up to 32; slices, or whole blocks with whole_blocks = 1;
                             3 = one workgroup per leaf box (leaf stages only, FP32 or FP64,
                             leaf sizes 4, 8, 16), one wave, or four with whole_blocks = 1:
                             the box or the padded fine block, the padded matrices and the
                             ranks requested in one memory round trip */
} tb_launch_cfg;

/* Set the configuration of launch `slot` for applies of p with exactly this
 * (nrhs, io) (manual tuning; tests force every candidate this way).  Slots
 * of the forward sequence: 0 .. Lt = source leaf and transfers (levels
 * 0 .. Lt), Lt + 1 = core, then target transfers and leaf (levels Ls .. 0);
 * the adjoint sequence follows at offset Lt + Ls + 3: target levels
 * 0 .. Ls, core, source levels Lt .. 0 (Lt, Ls from tb_plan_info).  Other
 * slots of a (nrhs, io) without an entry keep the heuristic.  Out-of-range
 * fields are TB_ERR_INVALID_ARG; a configuration that does not fit its
 * launch makes that apply fail with TB_ERR_UNSUPPORTED. */
tb_status tb_plan_set_launch(tb_plan p, long long nrhs, tb_dtype io, int slot, const tb_launch_cfg* cfg);

/* Fill *info.  Host only; no device work. */
tb_status tb_plan_info(tb_plan p, tb_plan_info_t* info);

/* Write / read the plan file (format below).  Save synchronises the device
 * (cores are copied back); load synchronises once it has uploaded.  Load
 * takes the cores from the file when it holds them, otherwise evaluates
 * them on the GPU; recompute_cores = 1 always evaluates them on the GPU.
 * opt supplies store_mask and max_device_bytes (NULL -> defaults). */
tb_status tb_plan_save(tb_plan p, const char* path);
tb_status tb_plan_load(const char* path, const tb_options* opt,
                       int recompute_cores, void* hip_stream, tb_plan* out);

/* Release a plan and everything it owns (NULL is ignored).  Synchronises
 * the device before freeing. */
void tb_destroy(tb_plan p);

/* Kernel stages of the apply, for per-stage timing. */
typedef enum {
  TB_STAGE_SRC_LEAF = 0,      /* V: input blocks -> skeletons (forward)        */
  TB_STAGE_SRC_TRANSFER,      /* W: level l-1 -> level l (forward)            */
  TB_STAGE_CORE,              /* K(tbar, sbar) x F (forward)                  */
  TB_STAGE_TGT_TRANSFER,      /* P^T, summed into the parents (forward)       */
  TB_STAGE_TGT_LEAF,          /* U^T: skeletons -> output blocks (forward)    */
  TB_STAGE_TGT_LEAF_ADJ,      /* conj(U) (adjoint)                            */
  TB_STAGE_TGT_TRANSFER_ADJ,  /* conj(P) (adjoint)                            */
  TB_STAGE_CORE_ADJ,          /* K(tbar, sbar)^H (adjoint)                    */
  TB_STAGE_SRC_TRANSFER_ADJ,  /* W^H, summed into the parents (adjoint)       */
  TB_STAGE_SRC_LEAF_ADJ,      /* V^H (adjoint)                                */
  TB_NSTAGES
} tb_stage;

/* Per-stage timing.  While enabled, tb_apply and tb_apply_adjoint record a
 * HIP event pair around every kernel they launch, on the caller's stream.
 * tb_plan_stage_times waits for those events, adds their durations (ms) and
 * launch counts per stage into ms[TB_NSTAGES] and launches[TB_NSTAGES]
 * (either may be NULL) and clears the record.  Timing adds an event record
 * per launch; leave it disabled for throughput runs. */
tb_status tb_plan_set_timing(tb_plan p, int enable);
tb_status tb_plan_stage_times(tb_plan p, double* ms, long long* launches);

const char* tb_last_error(void);
const char* tb_status_string(tb_status s);

/* Plan file, version 1 (little endian, no padding between fields):
 *   char[8]    "TBPLAN01"
 *   int32[8]   kind, d, n, leaf, L, Lt, Ls, has_cores
 *   float64[5] omega, tol, radon_a, radon_b, radon_den
 *   float64[d][n] target coordinates, TB_KERNEL_NUDFT plans only
 *   source IDs, for l = 0..Lt, s (level Ls, flat), tau (level l, flat),
 *     k = 0..d-1, nu = 0..2^(Lt-l)-1:   int32 r, int32 c, int32 skel[r],
 *     complex128 X[r][c]
 *   target IDs, for l = 0..Ls, t (level Lt), nu (level l), k, tau < 2^(Ls-l):
 *     int32 r, int32 c, int32 skel[r], complex128 X[r][c]
 *   cores if has_cores, for t, s: complex128 C[R_T][R_S] (row-major)
 *   uint32 CRC-32 (IEEE) of all preceding bytes, uint32 0
 * A multi-set (b_1..b_d) at level l has flat index sum_k b_k 2^(l(d-1-k)).
 * skel holds global per-mode indices in pivot order; X (r x c) satisfies
 * A ~= A(:, J) X for the sampled unfolding; its columns are the leaf's
 * indices (l = 0) or the first child's skeleton then the second's. */

#ifdef __cplusplus
}
#endif

#endif /* TB_H */
