/*
 * bmhd.h -- C ABI of the MI355X block-adaptive ideal-MHD library (libbmhd.so).
 *
 * The library advances the explicit second-order finite-volume ideal-MHD update over every 8x8x8
 * block of one or more simulations on one GPU (the single-GPU solver of the paper, Sec. 3 and
 * Algorithm 2): ghost cells from neighbour blocks with restriction and prolongation at resolution
 * changes (Sec. 4.1-4.2), limited linear face reconstruction, Rusanov or HLLE fluxes, the Powell
 * divergence source (Eqs. 1-4), and a two-stage update under a CFL-limited global time step (Sec. 5.1,
 * 5.2).
 *
 * Conventions
 *   - Every device pointer is memory the caller owns (PyTorch tensors in the Python binding). The
 *     library never allocates device memory. Pointers must be 8-byte aligned; d_work 256-byte aligned.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream. Every call that takes
 *     a stream only enqueues work on it and returns; nothing is synchronised. bmhd_advance may run part
 *     of a stage (the blocks near a body) on a side stream that the grid owns, made to wait for
 *     `stream` by an event and joined back into `stream` by another before the call returns, so all of
 *     its work is ordered on `stream` as if it ran there (while `stream` is being captured into a
 *     graph, everything stays on `stream`).
 *   - State arrays are variable-major, U[8][n_blocks][8][8][8] (k, j, i with i fastest), float64.
 *     Conserved order: rho, rho*ux, rho*uy, rho*uz, Bx, By, Bz, e (total energy, Eq. 5, mu0 = 1).
 *     Primitive order: rho, ux, uy, uz, Bx, By, Bz, p. gamma = 5/3.
 *   - Blocks are indexed in the caller's order; the library never reorders them.
 *   - Return value: BMHD_OK (0) or a negative code; bmhd_last_error() gives a message (thread-local).
 *     Launch errors are returned immediately. Numerical faults (rho <= 0, p <= 0, non-finite) are
 *     counted on the device into the caller's fault counter.
 *   - A grid handle must not be used from two host threads at once, and two calls that use the same
 *     uploaded workspace must not run concurrently on different streams.
 */
#ifndef BMHD_H
#define BMHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BMHD_OK 0
#define BMHD_EINVAL (-1)       /* bad argument or descriptor */
#define BMHD_EHIP (-2)         /* a HIP runtime call failed */
#define BMHD_ENOMEM (-3)       /* host allocation failed, or the workspace is too small */
#define BMHD_EUNSUPPORTED (-4) /* option combination not implemented */

#define BMHD_BC_PERIODIC 0
#define BMHD_BC_OUTFLOW 1 /* zero gradient: both ghost layers copy the nearest interior cell */
#define BMHD_BC_INFLOW 2  /* ghost cells hold the conserved form of inflow_W */

#define BMHD_FLUX_RUSANOV 0
#define BMHD_FLUX_HLLE 1
#define BMHD_FLUX_LINDE 2 /* HLLE plus the anti-diffusion of the entropy (contact) wave: the flux the paper's
                             fast-wave test names (Sec. 5.1), here after Linde's two-state HLL solver (whose
                             aim is no HLL dissipation on an isolated intermediate discontinuity): the density
                             jump no pressure change explains, delta = minmod(drho - dp / c^2, drho) with
                             c^2 = gamma (p_L + p_R) / (rho_L + rho_R), carried at the mean velocity u_bar, is
                             upwinded at lambda = u_bar_n clamped to [S_L, S_R]: F = F_HLLE + delta (S_L
                             max(lambda, 0) + S_R min(lambda, 0) - S_L S_R) / (S_R - S_L) (1, u_bar, 0, 0, 0,
                             |u_bar|^2 / 2). An isolated contact gets the exact upwind flux. */

#define BMHD_FP64 0      /* every step in float64 */
#define BMHD_FP32_FLUX 1 /* reconstruction and fluxes in float32; update, flux correction, dt in float64 */
#define BMHD_SCHEME_FACE 1
#define BMHD_SCHEME_PLANE 2
#define BMHD_SCHEME_BLOCK 3
#define BMHD_AUTOTUNE_SHAPES 13 /* launch shapes bmhd_autotune times */

/* Neighbour relations reported by bmhd_grid_neighbors. */
#define BMHD_REL_SAME 0
#define BMHD_REL_COARSER 1
#define BMHD_REL_FINER 2
#define BMHD_REL_OUTFLOW (-1)
#define BMHD_REL_INFLOW (-2)

/* One simulation (an independent domain with its own root-block box and time step). */
typedef struct {
    int32_t nroot[3];     /* level-0 blocks per axis */
    double origin[3];     /* lower domain corner */
    double dx0;           /* level-0 cell size (level 1: dx0 / 2) */
    int32_t bc[6];        /* x-lo, x-hi, y-lo, y-hi, z-lo, z-hi: BMHD_BC_*; periodic must pair up */
    double inflow_W[8];   /* primitive inflow state */
    double body_c[3];     /* centre of the reflecting body */
    double body_r;        /* radius; <= 0 means no body. Cells whose centre lies strictly inside are
                             body cells: never updated, never in dt, reflecting faces */
} bmhd_sim_desc;

/* A grid of blocks over n_sims simulations. Block b has refinement level level[b] in {0, 1}, block
 * index ijk[3b..3b+2] at that level (level-1 indices are twice as fine) and simulation sim[b]. Every
 * root block must be either one level-0 block or exactly its 8 level-1 children. */
typedef struct {
    int32_t n_blocks;
    const int32_t *level; /* host [n_blocks] */
    const int32_t *ijk;   /* host [n_blocks][3] */
    const int32_t *sim;   /* host [n_blocks] */
    int32_t n_sims;
    const bmhd_sim_desc *sims; /* host [n_sims] */
} bmhd_grid_desc;

/* Learned flux correction inside bmhd_advance (uniform grids only). Per stage: the 4-cell stencil of
 * every face (primitives in the face-normal frame (rho, u_n, u_t1, u_t2, B_n, B_t1, B_t2, p), z-scored
 * with stats[0..63]) goes through the MLP; its output, de-normalised with stats[64..79] and rotated back,
 * is added to the face flux. Cells whose provisional state has rho <= 0 or p <= 0, or rho or p outside
 * [min - tau * h, max + tau * h] of their old 7-point neighbourhood (FP64 values of the stage input),
 * with h = max(max - min, floor_rel * max(|min|, |max|)), are flagged; every face of a flagged cell falls
 * back to the plain flux on both sides and the affected cells are recomputed once. The flux scheme (the
 * second-order scheme of Sec. 5.1 with HLLE or Rusanov) is the paper's; the correction is this library's
 * own form. */
typedef struct {
    int32_t hidden;              /* 32, 64 or 128 */
    int32_t mode;                /* 0: BF16 matrix cores, 1: FP32 reference, 2: no network: y_buf holds
                                    the normalised corrections as given (corrections from another source;
                                    params and x_buf may be NULL) */
    const float *params;         /* device [n_params] float32 */
    const uint16_t *params_bf16; /* device [n_params] bfloat16 copy */
    const float *stats;          /* device: in_mean[32], in_std[32], out_mean[8], out_std[8] */
    float *x_buf;                /* device scratch [n_blocks * 1728][32] float32; modes 0 and 1 store
                                    the features of every face once (the block's faces at positions 0..7
                                    along their normal, then the high face planes with no neighbour
                                    across them), mode 0 as bfloat16 in its first half (16-byte aligned) */
    float *y_buf;                /* device [n_blocks * 1728][8]: mode 2: the given corrections in
                                    bmhd_face_data's layout; modes 0 and 1: scratch (the network's
                                    outputs in the layout of x_buf) */
    uint8_t *flags;              /* device scratch [n_blocks * 512] */
    int32_t *fallback_cells;     /* device counter of flagged cells, incremented per stage (may be NULL) */
    double tau;                  /* tolerance of the neighbourhood bound (0.1) */
    double floor_rel;            /* least neighbourhood range, relative to its largest magnitude (>= 0;
                                    0: the range itself, which rejects any change where the old
                                    neighbourhood is uniform) */
} bmhd_learned;

typedef struct {
    int32_t flux;         /* BMHD_FLUX_* (the learned correction takes RUSANOV or HLLE) */
    int32_t powell;       /* 1: Powell source terms (right-hand sides of Eqs. 2-4) */
    int32_t precision;    /* BMHD_FP64 or BMHD_FP32_FLUX */
    int32_t recompute_dt; /* 1: dt = CFL-limited global minimum per simulation, recomputed at the start
                             of every step; 0: d_dt used as given for every step */
    double cfl;
    double alpha[2];      /* stage table: out = alpha U^n + (1 - alpha) U_in + beta dt L(U_in) */
    double beta[2];       /* Heun: alpha = {0, 0.5}, beta = {1, 0.5} */
    int32_t slab;         /* tile depth of the stage kernel: 0 = default, 4 or 8 cells along z */
    int32_t scheme;       /* work split of the stage kernel: 0 = default (BMHD_SCHEME_BLOCK, or
                             BMHD_SCHEME_PLANE when slab is 4, persist_wgs > 0 or the flux is
                             BMHD_FLUX_LINDE); BMHD_SCHEME_FACE: one face per
                             thread and direction, fluxes exchanged through LDS; BMHD_SCHEME_PLANE: one
                             wave per cell layer of the tile plus one wave for the tile's high-side faces,
                             fluxes exchanged across lanes (less LDS, more workgroups per CU);
                             BMHD_SCHEME_BLOCK: one workgroup of eight wavefronts per block, one wave per
                             cell layer, the block's high-side faces shared out over the eight waves (slab
                             0 or 8, persist_wgs 0) */
    int32_t persist_wgs;  /* 0: one workgroup per tile; > 0: a persistent grid of this many workgroups
                             (rounded up to a multiple of 8), each looping over tiles */
    int32_t use_graph;    /* 1: steps after the first replay one captured HIP graph of a whole step
                             (n_stages must be even; `events` are ignored) */
    const bmhd_learned *learned; /* NULL: plain fluxes */
    int32_t n_events;     /* length of `events`, or 0 */
    void **events;        /* optional caller-created hipEvent_t handles: when n_events >= 2 * n_stages,
                             events[2s] and events[2s+1] are recorded on `stream` right before and after
                             the stage kernel of stage s (for timing the dominant kernel; with the block
                             scheme they bracket the block-form launch, after the plane-form launch for
                             the blocks near a body) */
    int32_t local_dt;     /* 1: local time stepping (the steady-state sessions of Sec. 5.2): every fluid
                             cell advances with its own CFL step, dt_i = cfl * 1 / sum_d ((|u_d| + c_f,d) /
                             dx), in both stages and in the flux correction; d_dt is then one value per cell,
                             [n_blocks][8][8][8] like one variable of d_U (0 for body cells). Not combined
                             with `learned` (BMHD_EUNSUPPORTED). */
} bmhd_opts;

typedef struct {
    int32_t n_blocks;
    int32_t n_sims;
    int32_t n_level_faces;  /* block faces that border a different refinement level */
    int32_t n_flux_faces;   /* coarse block faces that get a flux correction */
    size_t work_bytes;      /* size of the device workspace bmhd_grid_upload needs */
} bmhd_grid_info;

typedef struct bmhd_grid bmhd_grid;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t bmhd_version(void);

/* Message of the last failing call on this thread ("" if none). Valid until the next call. */
const char *bmhd_last_error(void);

/* Validate a descriptor and build the host-side tables: the 26-direction neighbour table, the face
 * relations used for ghost filling (Sec. 4.2: copy, restriction, prolongation, boundary), the list of
 * coarse-fine faces for flux correction, and a Morton-ordered block schedule. Host only; no HIP call.
 * On success *out owns a handle the caller frees with bmhd_grid_destroy. Errors: BMHD_EINVAL for a
 * malformed descriptor (level outside {0,1}, block outside its root box, overlap, partial refinement,
 * unpaired periodic faces, non-positive cell size). Body cells are found from cell-centre positions,
 * ghost cells included, so a body is expected to stay clear of domain faces and resolution changes. */
int32_t bmhd_grid_create(const bmhd_grid_desc *desc, bmhd_grid **out);
void bmhd_grid_destroy(bmhd_grid *g);

/* Sizes of the tables bmhd_grid_create built (the grid information of Sec. 2 that the message passing of
 * Sec. 4.2 and 4.4 looks up per block and direction), and the device workspace they need. Host only.
 * Errors: BMHD_EINVAL for a null argument. */
int32_t bmhd_grid_info_get(const bmhd_grid *g, bmhd_grid_info *info);

/* The relation to the neighbour in each direction, the lookup Sec. 4.2 makes per block and direction
 * (same, finer or coarser resolution, or a domain boundary), as a neighbour table in host memory
 * h_out[n_blocks][26][5] (caller-owned): {relation, id0, id1, id2, id3} for the 26
 * directions (dx, dy, dz) in {-1,0,1}^3 \ {0}, enumerated with dx fastest. SAME/COARSER: id0 is the
 * neighbour. FINER: the finer blocks that touch the block, ordered x fastest over the free
 * sub-positions. OUTFLOW/INFLOW: the direction leaves the domain through a non-periodic face (the
 * first such axis in x, y, z order decides). Unused ids are -1. */
int32_t bmhd_grid_neighbors(const bmhd_grid *g, int32_t *h_out);

/* Send the tables built on the CPU to the GPU (Sec. 4.4 fills its maps on the CPU and sends them; Sec. 3.1
 * keeps everything the time loop reads resident on the GPU). Copies the tables into the caller's device
 * workspace d_work (work_bytes from bmhd_grid_info_get,
 * 256-byte aligned) on `stream`. The grid keeps d_work as a borrowed pointer: it must stay allocated
 * while the grid is used, and upload must be repeated if it moves. The host tables are read again
 * by the copy only until the stream reaches it (the call waits for the copy before returning). */
int32_t bmhd_grid_upload(bmhd_grid *g, void *d_work, size_t work_bytes, void *stream);

/* Primitive to conserved (Eq. 5) for every interior cell: d_U[8][nB][512] from d_W[8][nB][512]. */
int32_t bmhd_set_state(const bmhd_grid *g, const double *d_W, double *d_U, void *stream);

/* Every cell of every block including both ghost layers on faces, edges and corners, written into a
 * padded view d_view[8][nB][12][12][12] (interior copied). Ghost rules (Sec. 4.2): copy from an
 * equal-level neighbour; restriction (pairwise-tree mean of the 8 finer cells) from a finer one;
 * prolongation (coarse value plus a quarter of the minmod slope per axis toward the fine cell) from a
 * coarser one; periodic wrap, outflow copy of the nearest interior cell, inflow state. Bit-exact
 * (no contraction). */
int32_t bmhd_fill_ghosts(const bmhd_grid *g, const double *d_U, double *d_view, void *stream);

/* State of one grid moved onto another grid of the same simulations after a refinement change (Sec. 2:
 * a block is refined into its 8 children or 8 children are coarsened into their parent; Sec. 3 adapts the
 * grid on the CPU between steps and then rebuilds its message maps, which here is bmhd_grid_create and
 * bmhd_grid_upload of the new block list). Every cell of `to` takes the value the ghost rules of `from`
 * (as in bmhd_fill_ghosts) give at its level and global index: a copy where the block exists in both
 * grids, prolongation from the level-0 parent where a block was refined, restriction of the 8 children
 * where blocks were coarsened. d_U_from [8][from.n_blocks][512], d_U_to [8][to.n_blocks][512], both
 * caller-owned device memory, distinct. Bit-exact (no contraction). Both grids must be uploaded. Errors:
 * BMHD_EINVAL when the simulation descriptors differ or a block of `to` cannot be supplied that way. */
int32_t bmhd_remap(const bmhd_grid *from, const double *d_U_from, const bmhd_grid *to, double *d_U_to,
                   void *stream);

/* Training targets of the learned flux correction (this library's own form, not the paper's): for every
 * face of the level-0 grid `coarse`, the mean of the 4 face fluxes of `fine` (the same simulations with
 * every root refined once, all blocks level 1) that cover it minus the coarse face flux, per component:
 * d_T[coarse n_blocks * 1728][8] from d_Ff[fine n_blocks * 1728][8] and d_Fc[coarse n_blocks * 1728][8]
 * (float32 device buffers in the layout and face-normal frame of bmhd_face_data). The 4 fine faces are
 * averaged pairwise, ((f00 + f10) + (f01 + f11)) / 4 with the first tangential index fastest, in float64
 * without contraction, then rounded. Coarse blocks are restricted from the fine grid by bmhd_remap.
 * Errors: BMHD_EINVAL (grids not uploaded or not in that relation, null buffers). */
int32_t bmhd_face_targets(const bmhd_grid *fine, const float *d_Ff, const bmhd_grid *coarse, const float *d_Fc,
                          float *d_T, void *stream);

/* Refinement indicator per block into d_ind[n_blocks] (device): the largest normalised jump, over the
 * block's cells and the three axes, of the density and of |B|^2 between a cell's two face neighbours
 * (neighbours outside the block by the ghost rules of bmhd_fill_ghosts): |q+ - q-| / (q+ + q- + 1e-300).
 * The paper adapts its grid between steps on the CPU (Sec. 2-3) without stating a criterion; this is the
 * library's (bit-exact, no contraction). */
int32_t bmhd_block_indicator(const bmhd_grid *g, const double *d_U, double *d_ind, void *stream);

/* Host: the adapted block list for indicators h_ind[n_blocks] (host): a level-0 root whose indicator
 * reaches r_refine becomes its 8 level-1 children, a refined root whose 8 children all stay below r_coarsen
 * (<= r_refine) becomes one level-0 block, other roots keep their blocks (two levels, so the result is 2:1
 * balanced). The list runs over each simulation's roots with x fastest, a refined root listing its
 * children with x fastest: h_level[n], h_ijk[n][3], h_sim[n] (host, may be NULL to count only, else at
 * least max_blocks long), *n_out = n. Feed it to bmhd_grid_create, bmhd_grid_upload and bmhd_remap.
 * Errors: BMHD_EINVAL, BMHD_ENOMEM (max_blocks too small). */
int32_t bmhd_adapt(const bmhd_grid *g, const double *h_ind, double r_refine, double r_coarsen, int32_t *h_level,
                   int32_t *h_ijk, int32_t *h_sim, int32_t max_blocks, int32_t *n_out);

/* The CFL-limited time step (Sec. 5.1 runs at CFL 0.8, Sec. 5.2 at 0.6 and 0.85), reduced on the GPU so
 * that steps advance without a transfer to the host (Sec. 3.1): d_dt[n_sims] (device) = cfl * min over
 * fluid cells of 1 / sum_d ((|u_d| + c_f,d) / dx) from d_U (device, [8][n_blocks][8][8][8]), c_f,d the
 * fast magnetosonic speed along axis d. Errors: BMHD_EINVAL (null pointer, grid not uploaded, cfl <= 0). */
int32_t bmhd_reduce_dt(const bmhd_grid *g, const double *d_U, double cfl, double *d_dt, void *stream);

/* Advance n_stages stages of the two-stage scheme (Algorithm 2's block sweep, repeated). Stage s uses
 * table entry s % 2: even stages read d_U0 (with ghost cells from neighbours) and write d_U1; odd
 * stages read d_U1 and d_U0 and overwrite d_U0, so a whole step leaves U^{n+1} in d_U0. A call starts
 * at a step boundary; after an odd n_stages the intermediate state is in d_U1. d_dt[n_sims] (with
 * local_dt: d_dt[n_blocks * 512], one step per cell): with recompute_dt, dt is recomputed at the start of
 * every step (under local_dt by the first stage, from its input state) and d_dt returns the last step's
 * dt; otherwise d_dt is read as given. d_faults (int32[1], may be NULL) is incremented by the number of
 * fluid cells with rho <= 0, p <= 0 or a non-finite value at the end of each step. Requires a prior
 * bmhd_grid_upload. */
int32_t bmhd_advance(const bmhd_grid *g, double *d_U0, double *d_U1, double *d_dt, int32_t n_stages,
                     const bmhd_opts *opts, int32_t *d_faults, void *stream);

/* Per-face data of a state for training the learned correction. Faces are enumerated per block and
 * direction d: face f of direction d sits between cells f-1 and f along d; f runs over
 * (z * 8 + y) * 9 + x for d = 0, (z * 9 + y) * 8 + x for d = 1 and (z * 8 + y) * 8 + x for d = 2 (576 per
 * direction), so the global index is (b * 3 + d) * 576 + f (faces shared by two blocks appear twice,
 * with equal values). d_X (may be NULL) [n_blocks * 1728][32]: stencil features in the face-normal
 * frame, z-scored with d_stats[0..63] when d_stats is not NULL. d_F (may be NULL)
 * [n_blocks * 1728][8]: the plain numerical flux (MC reconstruction, `flux`, FP64 arithmetic) in the
 * face-normal frame (rho, (rho u)_n, (rho u)_t1, (rho u)_t2, B_n, B_t1, B_t2, e). */
int32_t bmhd_face_data(const bmhd_grid *g, const double *d_U, int32_t flux, const float *d_stats, float *d_X,
                       float *d_F, void *stream);

/* Autotuner: time every launch shape of the stage kernel (scheme FACE or PLANE, tile depth 4 or 8
 * cells, one workgroup per tile or a persistent grid of 2 or 4 workgroups per compute unit; scheme
 * BLOCK) for n_steps steps each with `base`'s other options, on the caller's buffers (they are advanced:
 * pass scratch copies), and write `base` with the fastest shape into *best. h_ms (host, may be NULL)
 * receives the milliseconds of the BMHD_AUTOTUNE_SHAPES (13) candidates: scheme FACE then PLANE, each in
 * the order (4,0) (4,2/CU) (4,4/CU) (8,0) (8,2/CU) (8,4/CU), then BLOCK. Blocking: synchronises `stream`. With the environment variable
 * BMHD_AUTOTUNE_CACHE naming a file, the choice is kept there, one text line per configuration keyed by
 * the device (architecture, CU count), the grid (sizes and a hash of its block list) and the options
 * that change the work; a later call with the same key returns the stored shape without timing (h_ms
 * entries then -1) and leaves the buffers untouched. */
int32_t bmhd_autotune(const bmhd_grid *g, double *d_U0, double *d_U1, double *d_dt, const bmhd_opts *base,
                      int32_t n_steps, bmhd_opts *best, float *h_ms, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Ghost-cell exchange between processes: the message passing of Sec. 4.2-4.4 (Algorithm 4; message types
 * of Sec. 4.2: copy from an equal-level neighbour, restriction computed by the finer sender, prolongation
 * computed by the coarser sender), at one GPU's shapes. Blocks are assigned to processes (rank[b]); process
 * r keeps its blocks, in ascending global id (the local index), in a padded view
 * d_view[8][n_local(r)][12][12][12] of conserved values with two ghost layers, like bmhd_fill_ghosts'
 * view. Messages to other processes go through one buffer per (sender, receiver) pair and pass: each
 * message is a header of n_C = 7 doubles (receiving block's local index, low corner i, j, k, high corner
 * i, j, k of its receive box, inclusive, in the receiver's padded coordinates -2..9) followed by the box's
 * cells, 8 values each (v fastest, then i, j, k). Its start offset is the previous message's start plus
 * n_C plus the previous message's 8 * cells; the messages of one buffer follow the counting order
 * (sending process's blocks in local order, each block's 26 directions with x fastest). Pass 1 carries
 * copies and restrictions, pass 2 the prolongations (computed from the coarse sender's ghost cells after
 * pass 1). Messages within one process are written straight into its view. Ghost cells outside the
 * domain are filled by their own process (level-0 blocks after pass 1, level-1 blocks after pass 2).
 * After both passes every process's view equals the matching blocks of bmhd_fill_ghosts' view bit for
 * bit. The sequence per pass: bmhd_xchg_pack for every process, the transfers (any device copy, or a
 * point-to-point transfer between GPUs), bmhd_xchg_unpack for every process. */
typedef struct bmhd_xchg bmhd_xchg;

/* Count the message maps of an assignment rank[n_blocks] (host, values in [0, n_ranks)) on the host
 * (the paper rebuilds them only when the grid changes, Sec. 4.4): which messages each process sends and
 * receives in each pass and their start offsets. The grid must outlive the handle. Errors: BMHD_EINVAL. */
int32_t bmhd_xchg_create(const bmhd_grid *g, const int32_t *rank, int32_t n_ranks, bmhd_xchg **out);
/* The same message maps for the sharded stage (bmhd_xchg_stage, Sec. 4.4's step on each process): the
 * views then hold only the ghost cells the stage reads from them (faces whose neighbour is on another
 * process or level) and what the packs of those messages read. Messages between blocks of one process
 * are limited to restrictions, prolongations and the pass-1 ghost cells of blocks that send
 * prolongations; bmhd_xchg_interior copies only the blocks that send; boundary cells are filled only
 * for blocks that send prolongations. Message list and buffer sizes equal bmhd_xchg_create's. */
int32_t bmhd_xchg_create_for_stage(const bmhd_grid *g, const int32_t *rank, int32_t n_ranks, bmhd_xchg **out);
void bmhd_xchg_destroy(bmhd_xchg *x);

/* h_nloc[n_ranks] (may be NULL): blocks per process. h_len[2][n_ranks][n_ranks] (may be NULL): doubles in
 * the buffer from process s to process r in pass p + 1 (0 for s == r); a sender's send buffer holds its
 * buffers to the receivers one after another in receiver order, a receiver's receive buffer the buffers
 * from the senders in sender order. *work_bytes (may be NULL): the device workspace bmhd_xchg_upload
 * needs. */
int32_t bmhd_xchg_sizes(const bmhd_xchg *x, int32_t *h_nloc, int64_t *h_len, size_t *work_bytes);

/* The message list in counting order, one row of 16 int64 per message: sending process, receiving
 * process, pass, index among the messages of that (sender, receiver, pass), start offset, sending block,
 * direction slot (direction * 4 + finer sub-block), receiving block, its local index, type (0 copy, 1
 * restriction, 2 prolongation), box low corner (3), box high corner (3). With h_out NULL returns the
 * number of rows; otherwise fills up to max_rows rows and returns their number (BMHD_ENOMEM when too
 * small). Host only. */
int64_t bmhd_xchg_messages(const bmhd_xchg *x, int64_t *h_out, int64_t max_rows);

/* Copy the maps into the caller's device workspace (256-byte aligned, work_bytes from bmhd_xchg_sizes);
 * it must stay allocated while the handle is used. Waits for the copy. The grid must be uploaded before
 * the calls below. */
int32_t bmhd_xchg_upload(bmhd_xchg *x, void *d_work, size_t work_bytes, void *stream);

/* Process r's view with its blocks' interior cells from the global state d_U[8][n_blocks][512]. */
int32_t bmhd_xchg_interior(const bmhd_xchg *x, int32_t r, const double *d_U, double *d_view, void *stream);

/* Pass `pass` (1 or 2) on the sending side: every message process s sends to other processes, headers
 * and values computed from s's view, into d_send (sum over r of h_len[pass-1][s][r] doubles). */
int32_t bmhd_xchg_pack(const bmhd_xchg *x, int32_t pass, int32_t s, const double *d_view, double *d_send,
                       void *stream);

/* Pass `pass` on the receiving side: the messages in d_recv (sum over s of h_len[pass-1][s][r] doubles)
 * placed into r's view by their headers, then r's messages between its own blocks, then its boundary
 * ghost cells of the level this pass completes. A message whose header disagrees with the counted map (a
 * damaged buffer) is skipped and counted into d_bad (int32[1], may be NULL). */
int32_t bmhd_xchg_unpack(const bmhd_xchg *x, int32_t pass, int32_t r, const double *d_recv, double *d_view,
                         int32_t *d_bad, void *stream);

/* One stage of the two-stage scheme (Algorithm 2's block sweep; stage in {0, 1} picks alpha/beta of the
 * options' table) for process r's blocks after both exchange passes (Sec. 4.4: each process then updates
 * its own blocks): ghost cells of faces whose neighbour is on another process or level are read from r's
 * padded view d_view, those of same-process neighbours and domain boundaries in place. d_Uin, d_U0 and d_Uout are the
 * grid's [8][n_blocks][8][8][8] states, of which only r's blocks are read (d_Uin's own cells, d_U0's
 * own cells in the second stage) and written (d_Uout); dt is given per simulation (d_dt, the minimum over
 * every process: bmhd_reduce_dt stands in for that reduction on one GPU); positivity faults of the second
 * stage go to d_faults (may be NULL). Blocks clear of a body run on the block form, the others on the
 * plane form (all on the plane form with BMHD_FLUX_LINDE); the scheme, slab and graph options are not
 * used. Faces on a level change record their fluxes for bmhd_xchg_flux_correct, which runs after every
 * process's stage (the fine side's records are in the one device's memory here; between GPUs they would
 * travel like the ghost messages). Errors: BMHD_EINVAL; BMHD_EUNSUPPORTED with a learned correction,
 * local time stepping or a persistent grid. */
int32_t bmhd_xchg_stage(const bmhd_xchg *x, int32_t r, int32_t stage, const double *d_view, const double *d_U0,
                        const double *d_Uin, double *d_Uout, const double *d_dt, const bmhd_opts *o,
                        int32_t *d_faults, void *stream);
/* The flux corrections of process r's coarse cells next to a finer block after that stage (the coarse
 * face flux replaced by the mean of the fine ones), as bmhd_advance applies them. */
int32_t bmhd_xchg_flux_correct(const bmhd_xchg *x, int32_t r, int32_t stage, double *d_Uout, const double *d_dt,
                               const bmhd_opts *o, int32_t *d_faults, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Learned flux correction: a multilayer perceptron 32 -> H -> H -> H -> 8 with SiLU activations
 * (hidden width H in {32, 64, 128}). This component is not in the paper: it corrects the plain flux
 * of a coarse grid toward that of a grid twice as fine. Parameters are one flat float32 vector W1[H][32], b1[H], W2[H][H], b2[H], W3[H][H], b3[H],
 * W4[8][H], b4[8] (row-major, output index first) plus a bfloat16 copy of it (uint16 storage) that the
 * matrix-core products read. Loss: mean over samples and the 8 outputs of the squared error.
 * mode 0: products on BF16 matrix cores with FP32 accumulation; mode 1: FP32 FMAs (reference mode).
 * All buffers are caller-owned device memory; calls are asynchronous on `stream`. */
const char *bmhd_mlp_last_error(void);
int64_t bmhd_mlp_n_params(int32_t hidden);
/* Bytes of the scratch buffer bmhd_mlp_backward needs for n samples. */
size_t bmhd_mlp_work_bytes(int32_t hidden, int32_t n);
/* y[n][8] = MLP(x[n][32]); with d_save (float [3][n][H], may be NULL) the three hidden
 * pre-activations are kept for the backward pass. */
int32_t bmhd_mlp_forward(const float *d_params, const uint16_t *d_params_bf16, int32_t hidden, int32_t n,
                         const float *d_x, float *d_y, float *d_save, int32_t mode, void *stream);
/* Gradient of the loss against targets d_t[n][8] into d_grad (n_params floats, overwritten), given the
 * forward's d_y and d_save; d_sqerr[n][8] receives the squared errors. Deterministic (no atomics). */
int32_t bmhd_mlp_backward(const float *d_params, int32_t hidden, int32_t n, const float *d_x, const float *d_t,
                          const float *d_save, const float *d_y, float *d_grad, float *d_sqerr, float *d_work,
                          int32_t mode, void *stream);
/* bmhd_mlp_backward without the d_work argument, for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid allocation): the work area is a static
 * device array of the library, 32 MiB per device, held until the process ends and looked up on each
 * device's first call. It calls no allocating routine. n is limited to 8,388,608 / (16 + 2 * hidden)
 * samples (104,857 at hidden 32; 58,254 at 64; 30,840 at 128); a larger n returns BMHD_EINVAL with a
 * message and launches nothing. Results equal bmhd_mlp_backward's. Every call on one device shares that
 * device's array: calls that overlap on one device (different streams or host threads) race. */
int32_t bmhd_mlp_backward_noalloc(const float *d_params, int32_t hidden, int32_t n, const float *d_x,
                                  const float *d_t, const float *d_save, const float *d_y, float *d_grad,
                                  float *d_sqerr, int32_t mode, void *stream);
/* One Adam step (step count t >= 1) on the float32 parameters; refreshes the bfloat16 copy. */
int32_t bmhd_mlp_adam(float *d_params, uint16_t *d_params_bf16, float *d_m, float *d_v, const float *d_grad,
                      int64_t n_params, float lr, float b1, float b2, float eps, int32_t t, void *stream);
/* Refresh the bfloat16 copy from the float32 parameters (round to nearest even). */
int32_t bmhd_mlp_to_bf16(const float *d_params, uint16_t *d_params_bf16, int64_t n_params, void *stream);

#ifdef __cplusplus
}
#endif
#endif
