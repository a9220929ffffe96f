/*
 * lbm.h - C ABI of the MI355X lattice Boltzmann collide-and-stream library.
 *
 * The library advances a 3-D lattice Boltzmann simulation (D3Q19 or D3Q27)
 * by the fused collide-and-stream time step of Latt, Coreixas & Beny,
 * "Cross-platform programming model for many-core lattice Boltzmann
 * simulation" (arXiv:2010.11751):
 *   - collision  f_out_k(x) = Omega_k(f(x))        (Sec. 2.1, Eq. collision_step)
 *   - streaming  f_k(x + c_k, t+1) = f_out_k(x, t)  (Sec. 2.1)
 *   - half-way bounce-back with momentum exchange   (Sec. 2.1, Eq. momentum-exchange)
 *     f_kbar(x, t+1) = f_out_k(x, t) - 6 t_k rho_w c_k . u_w, rho_w = 1,
 *     wall cells storing the precomputed term        (Eqs. storage1, storage2)
 *   - memory-access schemes 2Pop / swap / AA        (Sec. 2.3, Table 1)
 *     and 2Pop in pull form (below)
 *   - layouts SoA pop[k][N] and AoS pop[N][Q]       (Sec. 2.3)
 *   - collision models BGK, TRT, regularized, recursive regularized, and the
 *     moment-space models of Sec. 2.2 (BGK with the non-weighted fourth-order
 *     equilibrium; multi-relaxation-time in raw, Hermite, central, central
 *     Hermite moments and cumulants, Sec. 2.6 Eq. RMcoll), with the
 *     bulk-viscosity knob of Sec. 2.6 (Eq. bulk).
 * The handle plays the role of the paper's stateless per-cell operator over
 * a lattice pointer, velocities, weights, omega and dimensions (Sec. 2.5).
 *
 * Conventions
 *   - Cell (x, y, z) has linear index i = (x*ny + y)*nz + z (z fastest), as
 *     in Sec. 2.5; Ntot = nx*ny*nz; every index is 64-bit safe.
 *   - Velocity order (D3Q19): k = 0..8 are (-1,0,0) (0,-1,0) (0,0,-1)
 *     (-1,-1,0) (-1,0,-1) (-1,0,1) (-1,1,0) (0,-1,-1) (0,-1,1); k = 9 is rest;
 *     c_{k+10} = -c_k. D3Q27: k = 0..12 are the same nine followed by
 *     (-1,-1,-1) (-1,-1,1) (-1,1,-1) (-1,1,1); k = 13 is rest; c_{k+14} = -c_k.
 *     This order has c_0 = (-1,0,0) = -c_10 as in the worked example of Sec. 2.6.
 *   - "Natural populations" f[k][Ntot] (FP64) are the pre-collision values of
 *     Eq. storage1 in every fluid cell and the stored momentum-exchange terms
 *     in wall cells, whatever the scheme, layout, AA phase or storage type.
 *   - Flags (uint8): LBM_FLUID, LBM_WALL, LBM_LID. Cavity geometry: fluid
 *     inside, one wall layer on each face, the whole z = nz-1 layer is the lid
 *     moving with lid_velocity. Periodic: all fluid, all axes wrap. Channel:
 *     x and y wrap, wall at z = 0, lid at z = nz-1.
 *   - Pointers are device pointers unless lbm_desc.ptr_kind = LBM_PTR_HOST.
 *   - Every call is ordered on the handle's stream; calls that return data to
 *     the caller (macroscopic, populations, flags, invariants) wait for it.
 *   - A handle is not thread safe. Errors: negative return codes, NULL
 *     handles; lbm_last_error() gives the thread's last message.
 *
 * Performance switches (read at handle creation; none changes any result):
 *   LBM_STRIDE_PAD=n        fixed SoA stride padding of n elements (0..3072)
 *                           instead of timing the candidates (lattices of
 *                           2^21 cells and more time 0, 256, 1024, 3072)
 *   LBM_STEP_LDS=a[,b]      fixed dynamic LDS bytes per block of the fast step
 *                           kernels of local / neighbour kinds, replacing the
 *                           residency cap chosen by storage type
 *   LBM_NO_RESIDENCY_CAP    no residency cap
 *   LBM_NO_GRAPH            no captured step graphs for small lattices
 *   LBM_PULL_KERNEL=box|flag  the 2Pop pull step on the built-in cavity or
 *                           periodic box: "box" the kernel that takes its
 *                           wall and wrap decisions from the cell's position,
 *                           "flag" the one driven by the flag byte and the
 *                           edge-cell list; unset, the one measured faster for
 *                           the lattice, storage type and layout
 *   LBM_AA_KERNEL=box|flag  the same for the AA odd step
 *   LBM_SPLIT_STEP          the edge-cell part as a second kernel on a second
 *                           stream instead of the leading blocks of the step
 *                           kernel
 *   LBM_NO_OVERLAP          with LBM_SPLIT_STEP: the edge-cell kernel on the
 *                           handle's stream
 *   LBM_VERBOSE             print the stride trials to stderr
 *   LBM_REVERSE_BLOCKS      step kernels visit the cells in reverse block and
 *                           list order (a traversal-order check: every
 *                           scheme is independent of it, Sec. 2.3)
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum lbm_status {
    LBM_OK = 0,
    LBM_EINVAL = -1,       /* bad argument (message in lbm_last_error)        */
    LBM_ENOMEM = -2,       /* device allocation failed                        */
    LBM_EDEVICE = -3,      /* HIP runtime error (HIP message attached)        */
    LBM_ENONFINITE = -4,   /* invariant monitor found NaN/Inf                 */
    LBM_EUNSUPPORTED = -5  /* valid but unsupported combination               */
};
/* LBM_2POP, LBM_SWAP and LBM_AA are the three schemes of Sec. 2.3 (Table 1;
 * 2Pop pushes each f_out_k to its neighbour). LBM_2POP_PULL is the
 * two-population scheme in pull form, not in the paper: between steps the
 * arrays hold post-collision values in slot kbar, as the AA pattern does after
 * an even step, and a step gathers f_k(x) from pop_kbar(x - c_k) (or
 * pop_k(x) + pop_kbar(x - c_k) across a wall), collides and stores
 * out_kbar(x) <- f_out_k at the cell's own index. The first step from a
 * pre-collision state (creation, lbm_init_equilibrium, lbm_set_populations)
 * is an AA even step. Its shifted accesses are reads, not writes. Results are
 * identical to the other schemes; read-outs apply the pending gather. */
enum lbm_scheme { LBM_2POP = 0, LBM_SWAP = 1, LBM_AA = 2, LBM_2POP_PULL = 3 };
/* BGK: BGK with the weighted second-order equilibrium (BGK-W2). TRT: two
 * relaxation times (Lambda). REG / RR: regularized and recursive regularized
 * (weighted Hermite). The moment-space models use the non-weighted basis of
 * Q moments (multi-indices in {0,1,2}^3; D3Q19 drops those with three nonzero
 * entries) and relax X*_n = X_n - w_n (X_n - X^eq_n) (Sec. 2.6, Eq. RMcoll):
 *   LBM_BGK_NW4  BGK with the non-weighted fourth-order equilibrium
 *   LBM_RM       raw moments          LBM_HM   Hermite moments
 *   LBM_CM       central moments      LBM_CHM  central Hermite moments
 *   LBM_K        cumulants (D3Q19 only; fourth-order cumulants relax)
 * with w = omega (second order, trace at omega_bulk per Eq. bulk), omega3
 * (third order) and omega4 (fourth order and up). All of them start from
 * and keep the NW4 equilibrium as their fixed point. */
enum lbm_collision {
    LBM_BGK = 0, LBM_TRT = 1, LBM_REG = 2, LBM_RR = 3,
    LBM_BGK_NW4 = 4, LBM_RM = 5, LBM_HM = 6, LBM_CM = 7, LBM_CHM = 8, LBM_K = 9
};
enum lbm_dtype { LBM_F64 = 0, LBM_F32_SHIFTED = 1, LBM_F16_SHIFTED = 2 };
/* LBM_SOA pop[k][N] and LBM_AOS pop[N][Q] are the layouts of Sec. 2.3.
 * LBM_BLOCKED keeps the Q streams of each run of 256 cells together (value
 * (k, i) at ((i / 256) Q + k) 256 + i mod 256, after whole blocks of padding):
 * an array-of-structures-of-arrays that keeps every stream access of a wave
 * contiguous while a block of cells touches one contiguous region; population
 * arrays of at most 4 GiB. Results are identical in every layout. */
enum lbm_layout { LBM_SOA = 0, LBM_AOS = 1, LBM_BLOCKED = 2 };
enum lbm_geometry { LBM_CAVITY = 0, LBM_PERIODIC = 1, LBM_CHANNEL = 2 };
enum lbm_flag { LBM_FLUID = 0, LBM_WALL = 1, LBM_LID = 2, LBM_PRESSURE = 3 };
enum lbm_ptr_kind { LBM_PTR_DEVICE = 0, LBM_PTR_HOST = 1 };

typedef struct lbm_handle lbm_handle;
typedef struct lbm_batch lbm_batch;

/* Full description of a simulation. Fill with lbm_desc_default() first. */
typedef struct lbm_desc {
    int lattice;          /* 19 or 27                                          */
    int nx, ny, nz;       /* box size, wall layers included                    */
    int scheme;           /* lbm_scheme                                        */
    int collision;        /* lbm_collision                                     */
    int storage_dtype;    /* lbm_dtype: FP64, or shifted g = f - t_k in FP32/FP16 */
    int layout;           /* lbm_layout                                        */
    int geometry;         /* lbm_geometry                                      */
    int ptr_kind;         /* lbm_ptr_kind of the data pointers of later calls  */
    int check_every;      /* >0: invariant monitor every so many steps         */
    int block_size;       /* threads per block of the step kernels; 0 = auto   */
    double omega;         /* shear relaxation frequency, 0 < omega < 2         */
    double trt_lambda;    /* TRT magic parameter (default 1/4)                 */
    double omega_bulk;    /* bulk relaxation of REG/RR/moment-space models;
                             <= 0 means = omega                                */
    double omega3;        /* moment-space models: rate of the third-order
                             moments; <= 0 means 1 (equilibrate)               */
    double omega4;        /* moment-space models: rate of the fourth- and
                             higher-order moments; <= 0 means 1                */
    double lid_velocity[3]; /* u_w of LID cells, |u_w| < 0.4                   */
    void *stream;         /* hipStream_t; NULL = the null stream               */
    void *pop;            /* optional caller-owned device buffers (see         */
    void *out;            /*   lbm_required_bytes); caller keeps ownership and */
    void *flags;          /*   must keep them alive until lbm_destroy          */
    size_t pop_bytes;     /* sizes in bytes of the caller buffers above; each  */
    size_t out_bytes;     /*   given buffer must hold at least what            */
    size_t flags_bytes;   /*   lbm_required_bytes reports, else LBM_EINVAL     */
} lbm_desc;

/* Per-handle facts for reporting. */
typedef struct lbm_info {
    int64_t ntot;             /* cells                                         */
    int64_t fluid_cells;      /* cells updated per step                        */
    int64_t pop_stride;       /* SoA elements between populations              */
    int64_t steps_done;       /* steps advanced since creation / last set      */
    int64_t first_nonfinite;  /* step at which the monitor tripped, else -1    */
    int64_t bytes_per_update; /* algorithmic HBM bytes per fluid-cell update    */
    int aa_phase;             /* AA: 1 if the next step is odd; 2Pop pull: 1
                                 once the state is post-collision            */
    int block_size;           /* block size the step kernels use               */
} lbm_info;

/* Fill d with defaults: D3Q19, 8^3 cavity, AA, BGK, FP64, SoA, omega 1,
 * Lambda 1/4, omega_bulk = omega, lid at rest, device pointers. */
void lbm_desc_default(lbm_desc *d);

/* Bytes of the population array(s) and flag array the description needs:
 * out[0] = pop, out[1] = out (0 unless 2Pop or 2Pop pull), out[2] = flags. Caller buffers
 * must be at least this large and 256-byte aligned. Returns a status. */
int lbm_required_bytes(const lbm_desc *d, size_t out[3]);

/* Create a cavity simulation (Sec. 3.1 benchmark case): lid moving along +x
 * at u_lid on the z = nz-1 layer; SoA; Lambda 1/4; omega_bulk = omega; null
 * stream; library-owned buffers. Initialised to equilibrium rho = 1, u = 0.
 * Returns NULL on error (see lbm_last_error). */
lbm_handle *lbm_create(int lattice, int nx, int ny, int nz, int scheme, int collision,
                       double omega, double u_lid, int storage_dtype);

/* Create from a full description; same initial state as lbm_create. Caller
 * buffers (pop, out, flags) are checked before any device work: each must be
 * 256-byte aligned and its size field (pop_bytes, out_bytes, flags_bytes) at
 * least what lbm_required_bytes reports; otherwise NULL with LBM_EINVAL (the
 * library never writes past a caller buffer it was told the size of). */
lbm_handle *lbm_create_ex(const lbm_desc *d);

/* Free library-owned buffers and the handle (caller buffers are untouched). */
void lbm_destroy(lbm_handle *h);

/* Set every fluid cell to the model's equilibrium E(rho, u) (Eq. storage1)
 * and every wall cell to its momentum-exchange terms (Eq. storage2).
 * rho[Ntot] and u[3][Ntot] (SoA) may be NULL (rho = 1, u = 0). Resets the
 * AA phase and the step counter. */
int lbm_init_equilibrium(lbm_handle *h, const double *rho, const double *u);

/* Replace the geometry by caller cell types (Sec. 2.1: link-wise bounce-back
 * Dirichlet walls with the momentum-exchange term of Eq. momentum-exchange,
 * stored in the wall cells as Eq. storage2). type[Ntot] holds LBM_FLUID,
 * LBM_WALL, LBM_LID or LBM_PRESSURE per cell (LID is a wall like any other
 * here). Each wall cell stores -6 t_k rho_w c_k . u_w from its own wall
 * velocity wall_velocity[3][Ntot] (SoA; NULL: at rest) and wall density
 * wall_density[Ntot] (NULL: 1); values of fluid cells are ignored.
 * LBM_PRESSURE cells are density (pressure) walls: a population reaching one
 * comes back with the opposite sign plus the stored term
 * 2 t_k rho_w [1 + 9/2 (c_k . u_w)^2 - 3/2 |u_w|^2] (anti-bounce-back, the
 * wall density set half-way along the link), in every scheme. The box
 * faces of axes that do not wrap (all of them for LBM_CAVITY, z for
 * LBM_CHANNEL) must be walls; |u_w| < 0.4 and 0 < rho_w < 10. Otherwise
 * returns LBM_EINVAL and leaves the handle unchanged. On success the fluid
 * cells are reset to E(1, 0), the AA phase and step counter to zero, and
 * later lbm_init_equilibrium calls keep these wall terms. Pointers follow
 * ptr_kind; the caller keeps ownership. */
int lbm_set_geometry(lbm_handle *h, const uint8_t *type, const double *wall_velocity,
                     const double *wall_density);

/* Curved walls (Sec. 1.1: the link-wise bounce-back extends to curved walls
 * while staying local). q[k][Ntot] (FP64, follows ptr_kind) gives, for every
 * fluid cell x and direction k whose upstream cell x - c_k is a wall (not a
 * pressure wall), the fraction 0 < q <= 1 of the link from x at which the
 * wall lies; other entries are ignored but must lie in (0, 1] too. The
 * population entering x is then the linear interpolated bounce-back
 *   q >= 1/2: [f_out_kbar(x) + (2q - 1) f_out_k(x) + w_kbar] / (2q)
 *   q <  1/2: 2q f_out_kbar(x) + (1 - 2q) f_out_kbar(x + c_k) + w_kbar
 * (f_out_kbar(x) in place of f_out_kbar(x + c_k) when x + c_k is not fluid),
 * the half-way rule at q = 1/2. All of these are values a cell gathering its
 * own populations reads, so the rule needs the 2Pop pull scheme: other
 * schemes return LBM_EUNSUPPORTED unless every q is 1/2 (which restores the
 * plain rule). Out-of-range values: LBM_EINVAL, handle unchanged. The
 * populations are kept; the rule applies from the next step. */
int lbm_set_wall_distances(lbm_handle *h, const double *q);

/* Advance n >= 0 time steps (asynchronous on the handle's stream unless the
 * invariant monitor is on). AA phase is tracked, so any n is allowed.
 * Returns LBM_ENONFINITE if the monitor finds a non-finite mass or energy.
 * Lattices of at most 2^20 cells (monitor off) run whole groups of 64 steps
 * from a HIP graph captured on first use; results are the same bit for bit. */
int lbm_step(lbm_handle *h, int n);

/* Density rho[Ntot] and velocity u[3][Ntot] (FP64) of the natural state;
 * wall cells get rho = 0, u = 0. */
int lbm_macroscopic(lbm_handle *h, double *rho, double *u);

/* Natural populations f[k][Ntot] (FP64), decoded from the storage type. */
int lbm_get_populations(lbm_handle *h, double *f);

/* Natural populations of the listed cells only: f[j*Q + k] for cells[j],
 * j < n (FP64), so that large lattices can be checked on samples. Both
 * arrays follow ptr_kind; indices must lie in [0, Ntot). */
int lbm_get_populations_at(lbm_handle *h, const int64_t *cells, int n, double *f);

/* Load natural populations f[k][Ntot] (FP64) into fluid cells (wall-cell
 * entries are ignored: wall terms are fixed by the geometry). Encodes to the
 * storage type (round to nearest even), resets the AA phase to even. */
int lbm_set_populations(lbm_handle *h, const double *f);

/* Cell flags (LBM_FLUID / LBM_WALL / LBM_LID), flags[Ntot]. */
int lbm_get_flags(lbm_handle *h, uint8_t *flags);

/* Global mass sum_fluid sum_k f_k and kinetic energy 1/2 sum_fluid rho|u|^2
 * of the natural state, reduced in FP64 in a fixed order (host pointers). */
int lbm_invariants(lbm_handle *h, double *mass, double *kinetic_energy);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the global
 * mass and kinetic energy of lbm_invariants, computed by the same kernels in
 * the same order, with their partial sums in a fixed device array of the
 * library instead of per-handle memory. result[0] = mass, result[1] = kinetic
 * energy; result follows ptr_kind: a device pointer is written asynchronously
 * on the handle's stream (no wait), a host pointer is written before return.
 * Allocates nothing and calls no allocating routine. Limit: lattices of at
 * most 2^25 cells (larger ones return LBM_EINVAL); the array takes 2 MiB per
 * GPU for the life of the process. All calls on one GPU share that GPU's
 * array: calls whose executions overlap on one GPU (different streams, or
 * different threads) race and must be ordered by the caller. */
int lbm_invariants_noalloc(lbm_handle *h, double *result);

/* Linear index of the neighbour x + c_k of each listed cell, as the step
 * kernels compute it (wrapping on periodic axes): out[j*Q + k] for
 * cells[j], j < n. Both arrays follow ptr_kind. */
int lbm_neighbor_index(lbm_handle *h, const int64_t *cells, int n, int64_t *out);

/* Facts about the handle (host pointer). */
int lbm_get_info(lbm_handle *h, lbm_info *info);

/* Velocity table c[Q][3], weights t[Q], opposites opp[Q] of the kernels
 * (host pointers; no device needed). */
int lbm_lattice(int lattice, int32_t *c, double *t, int32_t *opp);

/* Plain device-to-device copy of `bytes` (multiple of 16, 16-byte aligned
 * pointers) by a streaming kernel on `stream` (hipStream_t, may be NULL).
 * Not part of the method: it measures the attainable HBM bandwidth that the
 * step kernels are compared with, and calibrates hardware byte counters. */
int lbm_device_copy(void *dst, const void *src, size_t bytes, void *stream);

/* Copy of nstreams (19 or 27) FP64 streams of n values each, stream s at
 * element offset s * stride of src and dst (device pointers, 8-byte aligned;
 * stride >= n, n < 2^32), one value of every stream per thread: all loads of
 * a thread issued before its stores, blocks of 256 threads asking for
 * lds_bytes (0..65536) of unused dynamic LDS to cap residency, on `stream`.
 * With ny = nz = 0 value i of every stream is copied in place; with both >= 1
 * stream s is read at i - d_s and written at i + d_s, d_s = (c_sx ny + c_sy)
 * nz + c_sz the offset of lattice velocity s (the AA odd step's pattern), and
 * both buffers must extend ny*nz + nz + 1 values before element 0 and after
 * the last stream. Not part of the method: the memory patterns of the step
 * kernels without their arithmetic, the ceilings they are compared with. */
int lbm_stream_copy(void *dst, const void *src, int nstreams, size_t n, size_t stride, int lds_bytes, int ny,
                    int nz, void *stream);

/* Memory-pattern probe over 19 FP64 streams of n values (not part of the
 * method: the access patterns of the step kernels without their arithmetic,
 * the ceilings they are compared with). Layout: block_log2 = 0 puts stream s
 * at element offset s * stride (SoA, stride >= n); block_log2 = 8 or 12 puts
 * the 19 streams of each block of 2^b cells together, value (s, j) at
 * ((j >> b) * 19 + s) * 2^b + (j & (2^b - 1)) (stride unused; n a multiple of
 * 2^b). pattern 0 reads and writes cell i; 1 reads stream s at i - d_s and
 * writes it at i (2Pop pull); 2 reads at i - d_s and writes at i + d_s (AA
 * odd), d_s = (c_sx ny + c_sy) nz + c_sz the offset of D3Q19 velocity s
 * (ny, nz >= 1 for patterns 1 and 2). vec = 1 or 2 consecutive values per
 * lane (2: SoA only; n a multiple of vec). Blocks of 256 threads ask for
 * lds_bytes (0..65536) of unused dynamic LDS to cap residency. Device
 * pointers to value (0, 0); with shifts both buffers must extend h values
 * before it and after the last value, h = ny*nz + nz + 1 (SoA) or
 * ceil((ny*nz + nz + 1) / 2^b) * 19 * 2^b (blocked), and 8-byte aligned
 * (16-byte for vec = 2 unshifted). Asynchronous on `stream` (hipStream_t,
 * may be NULL). */
int lbm_pattern_copy(void *dst, const void *src, size_t n, size_t stride, int block_log2, int pattern, int vec,
                     int lds_bytes, int ny, int nz, void *stream);

/* Wait for all work queued on the handle's stream. */
int lbm_sync(lbm_handle *h);

/* Message of the calling thread's last error ("" if none). */
const char *lbm_last_error(void);

/* ------------------------------------------------------------------------ */
/* Batched ensemble: many independent cubic or box cavities of uneven sizes
 * and relaxation frequencies advanced together, one kernel launch per time
 * step over a (cavity, tile) work table; the step loop can be captured in a
 * HIP graph. Each cavity is the same problem as lbm_create's. */

typedef struct lbm_cavity_desc {
    int nx, ny, nz;       /* wall layers included                              */
    double omega;         /* shear relaxation frequency                        */
    double u_lid;         /* lid speed along +x on the z = nz-1 layer          */
    double trt_lambda;    /* TRT magic parameter (<= 0: 1/4)                   */
} lbm_cavity_desc;

typedef struct lbm_batch_opts {
    int use_graph;        /* capture the step loop in a HIP graph              */
    int graph_steps;      /* steps per captured graph (even, default 100)      */
    int autotune;         /* time candidate launch shapes at creation: block
                             size x cells per thread, then the residency cap */
    int block_size;       /* fixed block size when autotune = 0 (0 = 256)      */
    void *stream;         /* hipStream_t; NULL = a library-owned stream        */
    const char *autotune_cache; /* text file of tuned launch shapes, one line
                             "key block cells_per_thread waves_per_simd xcd" per
                             ensemble (key: GPU arch, scheme, collision,
                             dtype, cavity sizes); a hit skips the trial runs,
                             a miss appends the result; NULL: none          */
    int cells_per_thread; /* fixed runs of block_size cells per block of the
                             fast kernel when autotune = 0: 1, 2 or 4 (0 = 1) */
    int waves_per_simd;   /* fixed residency cap of the fast kernel when
                             autotune = 0: -1 = the storage type's default,
                             0 = none, 1..8 = that many waves              */
    int xcd_split;        /* fixed tile order when autotune = 0: 0 or 1 =
                             the table dealt to the eight XCDs in contiguous
                             parts (one cavity's tiles share an L2), 2 =
                             blocks in table order                          */
} lbm_batch_opts;

/* Create count cavities (FP64 or shifted FP32/FP16, D3Q19, any collision;
 * omega_bulk = omega and, for the moment-space models, omega3 = omega4 = 1)
 * under the 2Pop, AA or 2Pop pull scheme (swap: LBM_EUNSUPPORTED). opts may
 * be NULL (then: no graph, no autotuning, blocks of 256, one run per block,
 * default residency). Initial state: rho = 1, u = 0. A step is one kernel
 * over a (cavity, tile) table that skips each cavity's x = 0 and x = nx-1
 * wall layers (tiles of the largest cavities first), and, for the kinds that
 * reach neighbours, one kernel over the fluid cells next to two or more
 * walls, on a second stream of the library. */
lbm_batch *lbm_batch_create(int count, const lbm_cavity_desc *d, int scheme, int collision,
                            int storage_dtype, const lbm_batch_opts *opts);
int lbm_batch_step(lbm_batch *b, int n);
/* Same n steps, one kernel launch per cavity per step (reference timing). */
int lbm_batch_step_sequential(lbm_batch *b, int n);
int lbm_batch_macroscopic(lbm_batch *b, int idx, double *rho, double *u);
int lbm_batch_get_populations(lbm_batch *b, int idx, double *f);
/* FP64 mass and kinetic energy of every cavity: mass[count], ke[count] (host). */
int lbm_batch_invariants(lbm_batch *b, double *mass, double *kinetic_energy);
/* Total cells, fluid cells and block size in use (host pointers). */
int lbm_batch_info(lbm_batch *b, int64_t *cells, int64_t *fluid_cells, int *block_size);
/* Launch shape of the fast kernel in use (block size, cells per thread,
 * residency cap: -1 default, 0 none; XCD split 1 on, 0 off) and the number
 * of fluid cells next to two or more walls (host pointers, each may be
 * NULL). */
int lbm_batch_launch_shape(lbm_batch *b, int *block_size, int *cells_per_thread, int *waves_per_simd,
                           int *xcd_split, int64_t *edge_cells);
int lbm_batch_sync(lbm_batch *b);
void lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
