/*
 * lbf.h -- C ABI of the MI355X (gfx950) fluctuating lattice Boltzmann
 * library: the collide-and-stream update with thermal noise of Duenweg,
 * Schiller & Ladd, "Statistical mechanics of the fluctuating lattice
 * Boltzmann equation" (arXiv:0707.1581), on the D3Q19 lattice (basis of
 * Table II) or the D2Q9 lattice (basis of Table I).
 *
 * What one step computes (per lattice site r, step count t), with q = 19,
 * d = 3 for D3Q19 and q = 9, d = 2 for D2Q9:
 *   1. modes m_k = sum_i e_ki n_i(r) of the q populations with the
 *      lattice's basis (Sec. III, Eq. modes with the unscaled basis);
 *   2. rho = m_0, j = (m_1 .. m_d) (Eqs. defrho, defj) and the equilibrium
 *      stress modes of Eq. derived_equil_distrib (the kinetic modes have no
 *      equilibrium part);
 *   3. for every non-conserved mode k = d + 1 .. q - 1
 *        m*_k = m_k^eq + gamma_k (m_k - m_k^eq) + sqrt(mu rho w_k (1 - gamma_k^2)) r_k
 *      (Eqs. updaterule and FDT, Sec. IV), with mu = kT / c_s^2 = 3 kT in
 *      lattice units (Sec. VI), w_k the basis normalisers, rho the local
 *      density and r_k unit Gaussians; conserved modes k <= d are unchanged;
 *   4. back-transform n*_i = a_i sum_k e_ki m*_k / w_k and push along the
 *      links, n_i(r + c_i, t + 1) = n*_i(r, t), on a periodic box (Eq. LBE).
 * Mode rates: D3Q19 gamma_4 = gamma_bulk, gamma_5..9 = gamma_shear,
 * gamma_10..15 = gamma_odd (third-order kinetic modes), gamma_16..18 =
 * gamma_even (fourth-order kinetic modes); D2Q9 gamma_3 = gamma_bulk,
 * gamma_4..5 = gamma_shear, gamma_6..7 = gamma_odd, gamma_8 = gamma_even.
 *
 * Velocity order i, D3Q19: 0 rest; 1..6 = +x -x +y -y +z -z; 7..18 =
 * (+1,+1,0) (-1,-1,0) (+1,-1,0) (-1,+1,0) (+1,0,+1) (-1,0,-1) (+1,0,-1)
 * (-1,0,+1) (0,+1,+1) (0,-1,-1) (0,+1,-1) (0,-1,+1); weights a_i = 1/3,
 * 1/18, 1/36 (Sec. II).  D2Q9: 0 rest; 1..4 = +x -x +y -y; 5..8 = (+1,+1)
 * (-1,-1) (+1,-1) (-1,+1); weights 4/9, 1/9, 1/36 (the three-speed weights
 * fixed by the isotropy conditions of Sec. II).  c_s^2 = 1/3 for both.
 *
 * Random numbers: Philox4x32-10 keyed on the seed with counter
 * (site, t mod 2^32, call, t >> 32), 24-bit uniforms cut from each three
 * consecutive output words (most significant first), Box-Muller on
 * consecutive uniform pairs (cos first), normal s -> mode d + 1 + s.  The
 * site is the linear index x + nx (y + ny z) within the lattice, so a
 * replica of a batch draws exactly the numbers of the same lattice run
 * alone.
 *
 * State: one caller-owned device buffer holding, for every population i and
 * site, the scaled deviation delta_i = (n_i - a_i rho0) / (a_i rho0) in the
 * storage type (fp32, fp16 or bf16), as q planes [i][z][y][x] (x fastest),
 * updated in place with the AA access pattern: at even t, n_i(r) is held in
 * plane i at site r; at odd t, n_i(r) is held in plane opp(i) at site
 * r - c_i (opp(i) is the index of -c_i).  Callers never need this: all
 * gathers return parity-resolved populations, moments and modes.
 *
 * Conventions of every call:
 *   - device pointers (d_*) are caller-owned, contiguous, 256-byte aligned
 *     device memory; the library never frees them;
 *   - the stream is the caller's hipStream_t passed as void*; every kernel
 *     of a context runs on it; only lb_check, lb_autotune and lb_copy_rate
 *     synchronise;
 *   - argument errors are detected before anything is enqueued (nothing is
 *     done); launch failures return LB_EDEVICE, after which the state and
 *     step count of that context are undefined (some of the requested steps
 *     may have run); lb_last_error() gives the message of the last failure
 *     on the calling thread;
 *   - a context is not thread-safe; separate contexts are independent.
 */
#ifndef LBF_H
#define LBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum lb_status {
  LB_OK = 0,
  LB_EINVAL = -1,       /* invalid argument; nothing enqueued            */
  LB_EDEVICE = -2,      /* HIP runtime or launch failure                 */
  LB_ESTATE = -3,       /* lb_check found NaN or rho <= 0 sites          */
  LB_EUNSUPPORTED = -4  /* valid request the library does not provide   */
};

/* Storage of the state.  LB_BF16 is meant for fluctuating runs (kT > 0):
 * without noise its 8-bit mantissa biases slowly varying fields (a
 * noiseless shear wave decays about 2% too slowly), so deterministic runs
 * should store fp16 or fp32; lb_init accepts it and leaves a warning in
 * lb_last_error(). */
enum lb_storage { LB_F32 = 0, LB_F16 = 1, LB_BF16 = 2 };

enum lb_lattice {
  LB_D3Q19 = 0, /* 19 velocities on a cubic lattice, basis of Table II            */
  LB_D2Q9 = 1   /* 9 velocities on a square lattice, basis of Table I (nz = 1)    */
};

enum lb_init_kind {
  LB_INIT_REST = 0,    /* n_i = a_i rho0                                          */
  LB_INIT_THERMAL = 1, /* every normalised mode an independent unit Gaussian:     */
                       /* n_i = a_i rho0 + sqrt(mu rho0 a_i) sum_k ehat_ki z_k    */
                       /* (Eqs. xdef, x_s); normals from Philox stream 1          */
  LB_INIT_FIELDS = 2,  /* n_i = n_i^eq(rho, u) by Eq. derived_equil_distrib from  */
                       /* d_fields (1 + d, nz, ny, nx) fp32 = rho, ux, uy[, uz]   */
  LB_INIT_KEEP = 3     /* keep the buffer's contents as the state at step t0      */
};

enum lb_thermal_modes {
  LB_THERMAL_ALL = 0,        /* noise on every non-conserved mode (the paper's    */
                             /* detailed-balance collision, Sec. IV)              */
  LB_THERMAL_STRESS_ONLY = 1 /* noise on the stress modes only: the earlier       */
                             /* model the paper contrasts (kinetic modes get no   */
                             /* noise, violating detailed balance, Sec. IV)       */
};

typedef struct {
  int32_t nx, ny, nz;     /* periodic box, each >= 1 (1 makes that axis trivial); */
                          /* nz = 1 for D2Q9; at most 2^32 - 1024 sites           */
                          /* (LB_EUNSUPPORTED above)                              */
  int32_t storage;        /* enum lb_storage                                      */
  double rho0;            /* > 0: reference density and deviation base            */
  double kT;              /* >= 0: mu = 3 kT; kT = 0 gives the deterministic update */
  double gamma_bulk;      /* each gamma in [-1, 1] (linear stability, Sec. IV)    */
  double gamma_shear;
  double gamma_odd;
  double gamma_even;
  uint64_t seed;          /* Philox key                                           */
  int32_t thermal_modes;  /* enum lb_thermal_modes                                */
  int32_t lattice;        /* enum lb_lattice (0 = D3Q19)                          */
} lb_params;

typedef struct lb_ctx lb_ctx; /* opaque, library-owned */

/* Bytes of the state buffer: q * nx * ny * nz * sizeof(storage); 0 if the
 * parameters are invalid. */
size_t lb_state_bytes(const lb_params* p);

/* Validate p and create a context that updates d_state on hip_stream.
 * Enqueues the initial state (init_kind) as the state at step count t0
 * (t0 >= 0); d_fields is required for LB_INIT_FIELDS and ignored otherwise.
 * The context stores p by value.  Its default schedule (lb_get_schedule)
 * depends on the state: an fp32 lattice of more than 256 MiB (D3Q19) or
 * 32 MiB (D2Q9) takes the fused two-step schedule when the device has room
 * for its second state buffer (and its z-planes, or D2Q9 rows, hold less
 * than 4 GiB per population), which lb_init then allocates (release it with
 * lb_set_schedule and fused = 0).  With LB_BF16 storage and kT = 0
 * it succeeds and leaves a warning in lb_last_error(). */
int lb_init(const lb_params* p, void* d_state, void* hip_stream, int32_t init_kind,
            const float* d_fields, int64_t t0, lb_ctx** out);

/* Enqueue nsteps >= 0 steps (collide with noise keyed on the current t,
 * then push).  Full chunks of steps are replayed from a HIP graph (launched
 * one by one instead when a replay would exceed 2^16 kernel launches:
 * graph_chunk times the number of replica groups). */
int lb_step(lb_ctx* ctx, int64_t nsteps);

/* Enqueue nsteps >= 0 propagation-only steps: the streaming half of
 * Eq. LBE with the identity collision (what every rate gamma_k = 1 and
 * kT = 0 would give up to rounding), n_i(r + c_i, t + 1) = n_i(r, t) for
 * every population, periodic.  The stored values are moved unchanged, so
 * the result is an exact permutation of the state.  The step count advances
 * as with lb_step, keeping the parity-resolved layout consistent (later
 * collisions draw the noise of the advanced counter).  On a batch every
 * replica moves.  Each step is one launch over the tiles of the current
 * schedule (one per replica group), with the memory accesses and cache
 * policy of the step kernel it replaces, so its duration is the
 * data-movement floor of that step.  Steps are launched one by one, never
 * from a graph replay. */
int lb_propagate(lb_ctx* ctx, int64_t nsteps);

/* Parity-resolved gathers into caller-owned fp32 device buffers, each laid
 * out (count, nz, ny, nx):
 *   lb_populations: q planes, n_i;
 *   lb_moments:     1 + d planes, rho, jx, jy[, jz] (Eqs. defrho, defj);
 *   lb_modes:       q planes, m_k = sum_i e_ki (n_i - a_i rho0), so m_0 =
 *                   rho - rho0 and m_1..d = j. */
int lb_populations(lb_ctx* ctx, float* d_out);
int lb_moments(lb_ctx* ctx, float* d_out);
int lb_modes(lb_ctx* ctx, float* d_out);

/* Synchronising health check: counts sites with a non-finite population or
 * rho <= 0 into *n_bad and writes the lattice sums (sum rho, sum jx, sum jy,
 * sum jz; sum jz = 0 on D2Q9) in fp64 to sums_out[4] (either pointer may be
 * NULL).  Returns
 * LB_ESTATE when *n_bad > 0. */
int lb_check(lb_ctx* ctx, int64_t* n_bad, double* sums_out);

/* Completed steps t (the state held is the post-stream state at t). */
int64_t lb_step_count(const lb_ctx* ctx);

/* Release a context (a batch, a single lattice or a view). */
void lb_destroy(lb_ctx* ctx);

const char* lb_strerror(int code);
/* Message of the last failure on the calling thread (or the warning of a
 * later lb_init that succeeded with one); never NULL. */
const char* lb_last_error(void);

/* Lattice parameters from physical ones (Sec. VI, choice of parameters).
 * Inputs, in one consistent unit system: lattice spacing b > 0, time step
 * h > 0, mass density rho > 0 (mass per volume, or per area in 2D), shear
 * and bulk viscosities eta > 0 and zeta > 0, and k_B T >= 0; p->lattice
 * must be set on entry and selects the dimension d (3 for D3Q19, 2 for
 * D2Q9).  With the sound speed c_s^2 = (1/3) b^2/h^2 of both lattices,
 *   eta_hat  = eta h / (rho b^2 / 3),   gamma_shear = (2 eta_hat - 1) / (2 eta_hat + 1),
 *   zeta_hat = zeta h / (rho b^2 / 3),  gamma_bulk  = (d zeta_hat - 1) / (d zeta_hat + 1),
 *   mu = k_B T h^2 / ((1/3) b^(d+2))  (mass per site per particle), and in
 * lattice units (b = h = 1, mass unit rho b^d): rho0 = 1 and kT = mu / (3 rho)
 * = k_B T h^2 / (rho b^(d+2)).  Writes rho0, kT, gamma_shear and gamma_bulk
 * into *p and leaves its other fields as they are.  Returns LB_EINVAL for
 * invalid inputs or an unknown p->lattice (nothing is written). */
int lb_params_from_physical(double b, double h, double rho, double eta, double zeta, double kBT,
                            lb_params* p);

/* ---- ensembles: many independent lattices, one launch per step (per replica group) ---- */

/* Bytes of the pool for nrep replicas: each replica's state rounded up to
 * 256 bytes, in order; 0 if any replica is invalid. */
size_t lb_batch_pool_bytes(const lb_params* reps, int32_t nrep);

/* Byte offset of replica r in the pool. */
size_t lb_batch_offset(const lb_params* reps, int32_t nrep, int32_t r);

/* Create an ensemble of nrep >= 1 replicas with their own box, rates,
 * temperature and seed (one storage type and one lattice for all), laid out in d_pool as by
 * lb_batch_pool_bytes.  init_kind: LB_INIT_REST, LB_INIT_THERMAL or
 * LB_INIT_KEEP (LB_INIT_FIELDS returns LB_EUNSUPPORTED). */
int lb_batch_init(const lb_params* reps, int32_t nrep, void* d_pool, void* hip_stream,
                  int32_t init_kind, int64_t t0, lb_ctx** out);

/* Advance every replica by nsteps; one kernel launch per step covers all
 * replicas (one per replica group when the schedule's group_mb is set), and
 * full chunks of steps are replayed from a HIP graph. */
int lb_batch_step(lb_ctx* batch, int64_t nsteps);

/* A non-owning context for replica r (gathers and lb_check only; its step
 * count is the batch's).  Release with lb_destroy before the batch. */
int lb_batch_view(lb_ctx* batch, int32_t replica, lb_ctx** view);

/* ---- launch schedule and autotuning ---- */

typedef struct {
  int32_t block;        /* threads per workgroup: 64, 128, 256 or 512          */
  int32_t order;        /* tile order: 0 replica order, 1 largest replica      */
                        /* first, 2 smallest replica first                     */
  int32_t graph_chunk;  /* steps per graph replay (>= 2, even)                 */
  int32_t xcd_remap[2]; /* per step parity [even, odd]: which XCD takes which  */
                        /* tile (workgroup i runs on XCD i % 8): 0 tile i;     */
                        /* 1 each XCD one contiguous eighth of the tiles;      */
                        /* g in 2..64 each XCD g consecutive tiles at a time   */
  int32_t tiling[2];    /* per step parity: 0 each workgroup takes `block`     */
                        /* consecutive sites; 1 each workgroup takes one       */
                        /* `block`-long segment of one x-row, so y/z offsets   */
                        /* are uniform (planes below 4 GiB, else               */
                        /* LB_EUNSUPPORTED)                                    */
  int32_t resident;     /* cache policy of the step kernels: 0 streaming (non- */
                        /* temporal accesses, except the odd step's x-shifted  */
                        /* planes); 1 every access cached, for state that      */
                        /* stays in the 256 MB Infinity Cache across launches  */
                        /* (planes below 4 GiB, else LB_EUNSUPPORTED)          */
  int32_t group_mb;     /* 0: every step is one launch over all lattices; g > 0 */
                        /* (up to 2^20): lattices in tile order are packed into */
                        /* groups of at most g MiB of state (a larger lattice  */
                        /* is a group of its own), each step launches once per */
                        /* group, and a graph replay runs all graph_chunk      */
                        /* steps of one group before the next.  Replicas are   */
                        /* independent, so results do not depend on it.        */
  int32_t fused;        /* 0: one in-place AA launch per step.  1: two steps   */
                        /* per launch: from even t, each launch reads the      */
                        /* state once and writes the state two steps later     */
                        /* into a second buffer that the library allocates     */
                        /* (the size of the state) and releases when the       */
                        /* schedule goes back to 0 or the context is           */
                        /* destroyed.  Pairs of launches return the state to   */
                        /* the caller's buffer, so between calls it is always  */
                        /* there; steps that do not fill a pair of launches    */
                        /* run as AA steps.  Results are bit-identical to      */
                        /* fused = 0.  Single lattices (D3Q19 or D2Q9) whose   */
                        /* z-planes (D2Q9: rows) hold less than 4 GiB per      */
                        /* population only (else LB_EUNSUPPORTED, as when the  */
                        /* second buffer cannot be allocated); the             */
                        /* tiling, remap and cache-policy fields then apply to */
                        /* those AA steps only.                                */
} lb_schedule;

int lb_get_schedule(const lb_ctx* ctx, lb_schedule* out);
int lb_set_schedule(lb_ctx* ctx, const lb_schedule* s);

/* Time every candidate schedule on a scratch copy of the state (the state
 * and step count of ctx are unchanged): every block size and tile order
 * with every (xcd_remap in {0, 1, 2, 4, 8}, tiling) pair, timed on even and
 * on odd steps separately (`steps` >= 2 launches of each parity), with the
 * streaming cache policy and one group.  The six fastest candidates of each
 * parity are then timed again in three interleaved rounds, and the choice
 * rests on those times: the block size and order whose fastest even and
 * odd (remap, tiling) choices sum lowest.  A second stage times that
 * schedule on whole graph replays (at least 2 * `steps` steps, three
 * interleaved rounds) with each cache policy and, for a batch, replica
 * groups of 0, 64, 128, 160, 192, 224 and 256 MiB, and keeps a variant
 * only if it is at least 1% faster than the first stage's choice; a single
 * lattice also tries the fused two-step schedule there (when the
 * device has room for its second buffer).  Applies the best schedule and
 * writes a JSON report (one object per first-stage candidate with its mean
 * even and odd step times, plus refined_even_ms / refined_odd_ms for the
 * re-timed ones; then one object per second-stage variant with its
 * resident, group_mb, fused and ms_per_step) into report (NUL-terminated,
 * truncated to report_len).  Allocates a scratch copy of the state for as
 * long as it runs; returns LB_EUNSUPPORTED, having changed nothing, when the
 * device's free memory cannot hold that copy.
 * Cache: when the environment variable LBF_TUNE_CACHE names a file, a
 * schedule tuned earlier for the same device, library build, lattice,
 * storage and replica boxes (and noise on or off) is read from it and
 * applied without timing (report: [{"cached":true,"key":...}]); otherwise
 * the tuned schedule is appended to it.  An unreadable or unwritable file
 * only disables the cache; concurrent writers append whole lines. */
int lb_autotune(lb_ctx* ctx, int32_t steps, char* report, size_t report_len);

/* ---- a step entry point that allocates nothing ---- */

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Advances
 * nrep lattices (1 .. LB_NOALLOC_MAX_REPLICAS; one storage type and one
 * lattice model) by nsteps >= 0 steps on hip_stream, exactly as
 * lb_batch_init(reps, nrep, d_pool, hip_stream, LB_INIT_KEEP, t0) followed by
 * lb_batch_step(nsteps) would (for nrep = 1 the same as lb_init with
 * LB_INIT_KEEP and lb_step), with no context.  d_pool holds the lattices as
 * laid out by lb_batch_pool_bytes / lb_batch_offset (one state buffer for
 * nrep = 1), each in the AA layout of step t0's parity (as the library left
 * it at step count t0); the caller owns it.  Launch shape: the default
 * schedule's block size, tilings and XCD remap, the streaming cache policy,
 * one launch per step over all lattices, no graph.
 * Memory: calls no allocating routine.  The descriptors, tile prefixes and
 * the step counter go into one static device array of the library (about
 * 23 KB, LB_NOALLOC_MAX_REPLICAS descriptors), which each GPU the library
 * runs on holds until the process ends and which keeps the last call's
 * contents; every call rewrites what it uses, in stream order, before its
 * steps.  Calls that overlap on one GPU (on different streams, or from
 * different threads) race on that array: serialise them.
 * Errors: nrep above LB_NOALLOC_MAX_REPLICAS returns LB_EUNSUPPORTED;
 * invalid lattices, pointers, t0 < 0 or nsteps < 0 return LB_EINVAL (nothing
 * enqueued); launch failures LB_EDEVICE.  Asynchronous: returns once the
 * work is enqueued. */
#define LB_NOALLOC_MAX_REPLICAS 64
int lb_step_noalloc(const lb_params* reps, int32_t nrep, void* d_pool, void* hip_stream, int64_t t0,
                    int64_t nsteps);

/* ---- calibration ---- */

/* The practical streaming ceiling of the device: copies `bytes` (a positive
 * multiple of 16) from d_src to d_dst (caller-owned, 256-byte aligned,
 * non-overlapping device buffers) with one float4 per lane and
 * non-temporal loads and stores, once as a warm-up and then `reps` >= 1
 * times on the given stream, timed with HIP events, and writes the rate
 * counting bytes read plus bytes written, in GB/s, to *gbs_out.
 * Synchronises the stream.  Not part of the method: a reference against
 * which the step kernels' HBM rate is read. */
int lb_copy_rate(const void* d_src, void* d_dst, size_t bytes, int32_t reps, void* hip_stream, double* gbs_out);

#ifdef __cplusplus
}
#endif

#endif /* LBF_H */
