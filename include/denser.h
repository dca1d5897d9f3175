/*
 * denser.h -- C ABI of the MI355X (gfx950) library for sparse TSDF fusion
 * into hashed 8^3 voxel blocks and the Omega-masked TV primal-dual
 * regulariser of "DENSER Cities: A System for Dense Efficient
 * Reconstructions of Cities" (Tanner, Pinies, Paz, Newman).
 *
 * Conventions shared by every call
 *  - Plain C types only.  "dev" pointers are HIP device memory owned by the
 *    caller; "host" pointers are ordinary host memory.  The library never
 *    keeps a caller pointer after the call returns, except that device
 *    inputs must stay valid until the volume's stream has reached the call.
 *  - All device work is ordered on the HIP stream given to dn_volume_create
 *    (or dn_set_stream).  Calls that must return a count or a status to the
 *    host synchronise that stream before returning; the others only enqueue.
 *  - The library never allocates device memory.  A volume lives in one
 *    arena of dn_volume_bytes(params) bytes that the caller allocates and
 *    passes to dn_volume_create (pool, hash table, fields, solver state and
 *    the scratch every later call needs, sized there from the params'
 *    limits); the batched solver and the network calls take a workspace of
 *    the size their *_bytes function gives.  Calls whose input exceeds a
 *    limit return DN_E_CAPACITY and change nothing.  The caller frees the
 *    arena after dn_volume_destroy.
 *  - The library keeps no device state between calls outside the arenas
 *    and workspaces; host-side caches (kernel choices of the tuners, one
 *    captured batch graph per device) are guarded by a mutex.  Calls on
 *    one volume must not overlap.
 *  - Return value: DN_OK (0) or a negative DN_E_* code; dn_last_error()
 *    gives a thread-local message for the last failure.  A failed call
 *    leaves the volume unchanged unless its comment says otherwise.
 *  - A voxel's linear index inside its block is x + 8 y + 64 z.  Per-voxel
 *    fields are block-major: field[block][512].  The dual field p is three
 *    planes: p[3][n_blocks][512].
 *  - Camera frame: x right, y down, z forward; pixel (x, y) has its centre
 *    at integer coordinates.  A pose T_gc is a row-major 4x4 float64 host
 *    array mapping camera coordinates to world (global) coordinates.
 */
#ifndef DENSER_H
#define DENSER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------- status codes */
#define DN_OK 0
#define DN_E_INVALID (-1)   /* bad argument (null pointer, size, parameter)   */
#define DN_E_CAPACITY (-2)  /* block pool, hash table or output too small     */
#define DN_E_NUMERIC (-3)   /* non-finite energy or gap                       */
#define DN_E_DEVICE (-4)    /* HIP runtime error                              */

/* ------------------------------------------------- storage of u, ubar, p */
#define DN_F32 0          /* 32-bit float state                                */
#define DN_F16 1          /* IEEE half state, FP32 arithmetic                  */
#define DN_BF16 2         /* bfloat16 state, FP32 arithmetic                   */

/* --------------------------------------------------- initial solver state */
#define DN_INIT_ZERO 0   /* u = ubar = p = 0 (Section III-C, step 1)          */
#define DN_INIT_KEEP 1   /* continue from the state the last call left        */
#define DN_INIT_GIVEN 2  /* u = ubar = u0_dev, p = p0_dev (p0 may be NULL: 0)  */
#define DN_INIT_CONTINUE 3 /* regularisation interleaved with fusion (Section II:
                              the map is continuously regularised): blocks that
                              a previous call regularised keep their state,
                              blocks allocated since start at u = ubar = f,
                              p = 0; the step schedule restarts               */

/* ------------------------------------------------------- kernel choices */
#define DN_K_AUTO 0      /* pick the measured-best variant (autotuned)        */
#define DN_K_TWOPASS 1   /* dual kernel then primal kernel, per iteration     */
#define DN_K_FUSED 2     /* one LDS-staged kernel per iteration, 512 threads  */
#define DN_K_FUSED256 3  /* the same with 256 threads, two voxels per thread  */

/* ----------------------------------------------------- dn_extract targets */
#define DN_X_COORDS 1     /* int32 [n_blocks][3] block keys, pool order        */
#define DN_X_HASH 2       /* int32 [cap + tail][4] slots {x, y, z, id}, id<0 empty */
#define DN_X_NBR 3        /* int32 [n_blocks][27] 3x3x3 neighbourhood ids       */
#define DN_X_F 4          /* float [n_blocks][512] fused TSDF f                */
#define DN_X_W 5          /* float [n_blocks][512] fusion weight w             */
#define DN_X_U 6          /* float [n_blocks][512] primal u (as float)         */
#define DN_X_UBAR 7       /* float [n_blocks][512] relaxed primal ubar          */
#define DN_X_P 8          /* float [3][n_blocks][512] dual p                   */
#define DN_X_SURFACE 9    /* float [n][3] zero crossings of u (world metres)   */
#define DN_X_CANDIDATES 10 /* int32 [n][3] distinct block keys the last
                              dn_alloc_blocks frame touched, ascending          */
#define DN_X_EMASK 11     /* uint8 [n_blocks][512] bit0 Omega, bit1+a m_a     */
#define DN_X_MESH 12      /* float [n][3][3] triangles of the zero level set of
                             u (world metres), see dn_extract                */

typedef struct dn_volume dn_volume;

typedef struct {
    double fx, fy, cx, cy;   /* pinhole intrinsics, pixels */
    int32_t width, height;   /* depth map size; the map is float32 row-major */
} dn_intrinsics;

typedef struct {
    double voxel_size;       /* s, metres (edge of a voxel)                  */
    double mu;               /* truncation distance, metres                  */
    double max_depth;        /* depths above this are treated as invalid     */
    int32_t max_blocks;      /* capacity of the block pool                   */
    int32_t hash_cap_log2;   /* the table has 2^hash_cap_log2 buckets ...    */
    int32_t hash_tail;       /* ... plus this many overflow slots            */
    int32_t state16;         /* 1: room for FP16/BF16 solver state (DN_F16,
                                DN_BF16 storage), 18 more bytes per voxel   */
    int64_t max_points;      /* most pixels of one depth map (width x height)
                                or returns of one laser scan a call takes
                                (0: the volume takes no sensor data)        */
    int64_t max_candidates;  /* most band cells (repeats counted) one
                                dn_alloc_blocks / dn_alloc_laser call may
                                list, and most keys of one dn_insert_blocks
                                call; a pixel's band crosses at most
                                4 + sqrt(3) 2 mu |r| / (8 s) blocks, r its
                                ray direction with unit depth              */
    int64_t max_observations; /* most voxel observations one dn_fuse_laser
                                call may make (0: no laser fusion)          */
} dn_volume_params;

typedef struct {
    double lambda;           /* data weight (Eq. 2)                          */
    double tau, sigma;       /* primal and dual step sizes (Eqs. 7-8)        */
    double theta;            /* relaxation (Eq. 9), 1 for the standard method */
    int32_t iters;           /* maximum number of iterations                 */
    int32_t gap_every;       /* compute the gap every this many iterations; 0: only at the end */
    double gap_tol;          /* stop once (E - D) / E <= gap_tol (0: never)  */
    int32_t storage;         /* DN_F32, DN_F16 or DN_BF16                    */
    int32_t refine_every;    /* 16-bit storage: FP32 sweep every this many iterations (0: none) */
    int32_t init;            /* DN_INIT_*                                    */
    int32_t kernel;          /* DN_K_*                                       */
    double gamma;            /* 0: fixed steps (tau, sigma, theta).  > 0: the
                                accelerated variant for a uniformly convex
                                data term with modulus gamma (lambda * min w
                                over Omega): theta_n = 1/sqrt(1 + 2 gamma
                                tau_n), tau_{n+1} = theta_n tau_n,
                                sigma_{n+1} = sigma_n / theta_n, starting
                                from (tau, sigma); the schedule continues
                                across calls with DN_INIT_KEEP           */
    int32_t data_term;       /* DN_DATA_L2: (lambda/2) w (u - f)^2 (Eq. 2 with
                                the weight of Eq. 8).  DN_DATA_L1: lambda w
                                |u - f| with u kept in [-1, 1] (the range of
                                the TSDF); its primal step is a soft threshold
                                of u~ - f by tau lambda w followed by the
                                clamp, its dual D(p) = sum over Omega of
                                min(-f d, -d + lambda w |1 - f|,
                                d + lambda w |1 + f|), d = div p.  The L1 term
                                is not uniformly convex: gamma must be 0.  */
} dn_reg_params;

#define DN_DATA_L2 0
#define DN_DATA_L1 1

typedef struct {
    double energy;           /* E(u), Eq. (2) with the weight of Eq. (8)      */
    double dual;             /* D(p), Eq. (6)                                 */
    double gap;              /* E - D  (>= 0 by weak duality)                 */
    double rel_gap;          /* (E - D) / E                                   */
    int32_t iters_run;       /* iterations performed by this call             */
    int32_t converged;       /* 1 if gap_tol was reached                      */
    double ms_loop;          /* HIP-event time of the iteration loop on the
                                volume's stream (gap checks included)        */
    int32_t kernel_used;     /* DN_K_* that ran (after autotuning)            */
    int32_t layout_used;     /* bit 0: pool order (else Morton order); bit 1:
                                plain workgroup map (else XCD chunks)        */
} dn_reg_stats;

/* ------------------------------------------------------------ lifecycle */

/* Bytes of device memory a volume with these parameters needs (its arena),
 * or 0 if the parameters are invalid.  Pure arithmetic: no device call. */
size_t dn_volume_bytes(const dn_volume_params *params);

/* Create an empty volume in the caller's arena.  hash_cap_log2 in [4, 30],
 * hash_tail >= 0, max_blocks >= 1, voxel_size > 0, mu > 0, max_depth > 0,
 * max_points, max_candidates, max_observations >= 0.  arena_dev: device
 * memory of arena_bytes >= dn_volume_bytes(params) bytes, 256-byte aligned,
 * owned by the caller and used by the volume until dn_volume_destroy.
 * hip_stream is a hipStream_t (NULL: the default stream).  *out receives
 * the handle.  DN_E_INVALID for bad parameters or a null or misaligned
 * arena, DN_E_CAPACITY for a short arena (both checked before any device
 * call). */
int dn_volume_create(const dn_volume_params *params, void *arena_dev, size_t arena_bytes, void *hip_stream,
                     dn_volume **out);

/* Release the handle (synchronises the volume's stream first).  The arena
 * is the caller's to free afterwards. */
void dn_volume_destroy(dn_volume *vol);

/* Remove every block (the volume becomes empty; its capacity is kept).
 * Enqueue only. */
int dn_volume_clear(dn_volume *vol);

/* Change the stream subsequent calls are ordered on. */
int dn_set_stream(dn_volume *vol, void *hip_stream);

/* Number of allocated blocks (host value; no synchronisation needed). */
int64_t dn_num_blocks(const dn_volume *vol);

/* Wait for all work enqueued on the volume's stream. */
int dn_sync(dn_volume *vol);

/* Thread-local text of the last error ("" if none). */
const char *dn_last_error(void);

/* ------------------------------------------------------------ allocation */

/* Block allocation for one depth map (Section III-A: a block is allocated
 * as soon as a surface is observed inside it).  Every valid pixel (finite,
 * 0 < d <= max_depth) marks every block that its ray crosses for depths in
 * [max(d - mu, 1e-3), d + mu] (a 3-D grid traversal over 8s-sized blocks;
 * ties step x, then y, then z).  Keys not yet present are appended to the
 * pool in ascending (x, y, z) order; existing pool ids never change.  The
 * hash table (Teschner primes, non-wrapping linear probing in ascending
 * (bucket, key) order) and the 27-neighbour table are rebuilt.
 * depth_dev: float32 [height][width].  T_gc: host float64[16].
 * *n_new_out (host, may be NULL) receives the number of new blocks.
 * DN_E_CAPACITY if width x height exceeds max_points, the band cells
 * exceed max_candidates, or the pool or the table would overflow (volume
 * unchanged).  Synchronises the stream. */
int dn_alloc_blocks(dn_volume *vol, const float *depth_dev, const dn_intrinsics *K,
                    const double T_gc[16], int32_t *n_new_out);

/* Append explicit block keys (int32 [n][3], device) with the same rules as
 * dn_alloc_blocks (duplicates and existing keys are ignored; new keys are
 * appended in ascending order).  n <= max_candidates (else DN_E_CAPACITY).
 * Synchronises the stream. */
int dn_insert_blocks(dn_volume *vol, const int32_t *coords_dev, int64_t n, int32_t *n_new_out);

/* dn_insert_blocks, except that the new keys are appended in the order of
 * their first occurrence in coords_dev (later repeats and keys already in
 * the volume are ignored), so the block pool holds them in the caller's
 * order: a map assembled from keys can keep the order in which fusion
 * (Section III-A) allocated its blocks, which decides how often a block's
 * halo is still in cache when its neighbours run.  n < 2^31 (else
 * DN_E_INVALID).  Synchronises the stream. */
int dn_insert_blocks_ordered(dn_volume *vol, const int32_t *coords_dev, int64_t n, int32_t *n_new_out);

/* --------------------------------------------------------------- fusion */

/* Projective TSDF update of every voxel of every allocated block with one
 * depth map, Eq. (1): p_c = T_gc^-1 p_g for the voxel centre (g + 0.5) s,
 * nearest pixel floor(X + 0.5), eta = d - z_c; if the pixel is inside the
 * map and valid and eta >= -mu: w += 1 and f = (min(1, eta/mu) + w_old f)/w.
 * Geometry and decisions in float64, f and w in float32.  Blocks that no
 * voxel centre of which can pass these tests (all behind the camera, all
 * beyond max_depth + mu, or projecting outside the image; a conservative
 * test on the block's corners) are skipped without reading their voxels,
 * so the cost of a frame follows the blocks in view, not the map; the
 * result is the same as updating every block.  Enqueue only. */
int dn_fuse_depth(dn_volume *vol, const float *depth_dev, const dn_intrinsics *K,
                  const double T_gc[16]);

/* Laser range data (Section III-A: the update extends to laser sensors by
 * updating only the voxels along each ray from the sensor to mu behind the
 * observed surface).  pts_dev: float [n][3] returns in the sensor frame,
 * T_gs row-major sensor-to-world (host).  A return's range is r = |p|,
 * valid iff finite and 0 < r <= max_depth, its direction p / r.
 * dn_alloc_laser: allocates the blocks that the band of range
 * [max(r - mu, 1e-3), r + mu] along each ray passes through (the same
 * traversal, append order and errors as dn_alloc_blocks).
 * dn_fuse_laser: every voxel of an allocated block that the ray meets
 * between the sensor and r + mu, with eta = r - (c - o) . D >= -mu (c the
 * voxel centre, o the sensor, D the world direction), observes
 * psi = min(1, eta / mu); one call applies all of its observations
 * together: f <- (w f + sum psi) / (w + k), w <- w + k (the sum in
 * float64).  Both synchronise.  DN_E_CAPACITY (volume unchanged) if n
 * exceeds max_points, the band cells max_candidates or the observations
 * max_observations. */
int dn_alloc_laser(dn_volume *vol, const float *pts_dev, int64_t n, const double T_gs[16], int32_t *n_new_out);
int dn_fuse_laser(dn_volume *vol, const float *pts_dev, int64_t n, const double T_gs[16]);

/* Overwrite f and w of all allocated blocks (device float [n_blocks][512]
 * each); w > 0 marks the voxel as observed (in Omega).  Enqueue only. */
int dn_load_fused(dn_volume *vol, const float *f_dev, const float *w_dev);

/* -------------------------------------------------------- regularisation */

/* Chambolle-Pock iterations on the masked TV + weighted quadratic energy
 * (Section III-B/C, Eqs. 2-9) over the allocated blocks:
 *   p = P(p + sigma grad ubar),  u' = prox(u + tau div p),
 *   ubar = u' + theta (u' - u),
 * with grad the forward differences of Eq. (3) that are zero unless both
 * voxels are observed (a voxel of an unallocated block is unobserved) and
 * div = -grad^T (Eq. 4).  Voxels outside Omega keep their u.
 * u0_dev (float [n_blocks][512]) and p0_dev (float [3][n_blocks][512]) are
 * read only with init == DN_INIT_GIVEN.  out_host (may be NULL) receives the
 * final energies.  DN_E_NUMERIC if the gap becomes non-finite.  16-bit
 * storage needs a volume created with state16 (else DN_E_INVALID).  A
 * 16-bit run leaves its result in the FP32 state as well (the output of its
 * last refinement sweep, or, when gap_tol stops it between sweeps, its
 * current state).  Synchronises the stream (at every gap check and at the
 * end). */
int dn_regularize(dn_volume *vol, const dn_reg_params *params, const float *u0_dev,
                  const float *p0_dev, dn_reg_stats *out_host);

/* Workspace bytes of dn_regularize_batch for n volumes holding
 * total_blocks blocks together (0 for bad arguments). */
size_t dn_regularize_batch_bytes(int32_t n, int64_t total_blocks);

/* Regularise n independent volumes with the same parameters in one HIP
 * graph, captured and replayed: either ONE persistent kernel launch (a
 * grid-wide barrier separates iterations) or one launch per iteration over
 * every volume: params->kernel DN_K_FUSED256 selects the latter, DN_K_AUTO
 * whichever the autotuner timed faster for this problem size (timed on the
 * first call of a size with init ZERO, the persistent kernel until then),
 * any other value the persistent kernel.  Work items are (volume, block) pairs balanced over the grid.
 * kernel_used of the stats: 100 x variant + workgroups per CU (variant 1:
 * one launch per iteration; 256 / 512: persistent with that many threads
 * per workgroup; 257: persistent, 256 threads, no prefetch).  All volumes must share one device; the
 * first volume's stream is used.  gap_every / gap_tol are ignored (the
 * gaps are computed once at the end); init must be ZERO or KEEP; storage
 * must be DN_F32.  workspace_dev: caller device memory of at least
 * dn_regularize_batch_bytes(n, sum of the volumes' blocks) bytes, 256-byte
 * aligned (else DN_E_CAPACITY / DN_E_INVALID); the captured graph refers to
 * it and is replayed while the same workspace, volumes and parameters come
 * back.  out_host: n stats (may be NULL). */
int dn_regularize_batch(dn_volume *const *vols, int32_t n, const dn_reg_params *params, void *workspace_dev,
                        size_t workspace_bytes, dn_reg_stats *out_host);

/* Primal and dual energies of the current state for the data term
 * data_term (DN_DATA_L2 or DN_DATA_L1): out_host[0] = E(u),
 * out_host[1] = D(p).  Synchronises. */
int dn_energy(dn_volume *vol, double lambda, int32_t data_term, double out_host[2]);

/* -------------------------------------------------------------- extract */

/* Copy a part of the volume (DN_X_*) into out_dev (device, out_bytes
 * long).  *n_out (host) receives the number of items (blocks, slots or
 * points).  If out_dev is NULL or too small, nothing is written, *n_out
 * still receives the count, and DN_E_CAPACITY is returned (for
 * DN_X_SURFACE the count is computed first).  Synchronises the stream.
 * DN_X_SURFACE: for every voxel g and axis a with both g and g + e_a
 * observed and a sign change (u < 0 differs), the point
 * (g + 0.5) s + t s e_a with t = u(g) / (u(g) - u(g + e_a)), in the order
 * (pool id, voxel index, axis).
 * DN_X_MESH (Section II: the surface model is the zero-crossing
 * isosurface; Tables III-IV report its area): triangles over every cube of
 * voxels g + {0,1}^3 whose eight corners are observed.  The cube (corner
 * k = x + 2y + 4z) is cut into six tetrahedra along its main diagonal,
 * corners 0, e_a0, e_a0 + e_a1, 7 for the axis orders (0,1) (0,2) (1,0)
 * (1,2) (2,0) (2,1); a vertex alone on its side of zero gives one triangle
 * on its three edges, two and two (negative a < b, positive c < d) give
 * (ac, ad, bd) and (ac, bd, bc); an edge point is P_i + t (P_j - P_i),
 * t = u_i / (u_i - u_j), from the corner with the smaller k; normals point
 * to u > 0.  Order (pool id, voxel, tetrahedron, triangle); float64
 * arithmetic rounded to float. */
int dn_extract(dn_volume *vol, int32_t what, void *out_dev, size_t out_bytes, int64_t *n_out);

/* Total area (float64, square metres) of the DN_X_MESH triangles and their
 * number (n_tris_host may be NULL).  Synchronises. */
int dn_mesh_area(dn_volume *vol, double *area_host, int64_t *n_tris_host);

/* ---------------------------------------------------- learned warm start */
/* The network: three 3x3x3 convolutions with "same" zero padding on a
 * 10^3 tile (a block plus a one-voxel halo): 2 -> 16 (ReLU) -> 16 (ReLU)
 * -> 1.  Inputs f and log(1 + w) / log(101); output r; the warm start is
 * u0 = clamp(f + r, -1, 1) on Omega.  Parameters are 8241 float32 values:
 * W1[16][2][27] b1[16] W2[16][16][27] b2[16] W3[1][16][27] b3[1], tap
 * (dz*3 + dy)*3 + dx.  Convolutions run on MFMA in bfloat16 with float32
 * accumulation (the layer-1 weights as the pair bf16(W) + bf16(W - bf16(W))). */
#define DN_NET_PARAMS 8241

/* Gather the input tiles of the listed blocks: float [n][2][10][10][10]
 * (channel, z, y, x).  perm exchanges the tile's x axis with the volume's
 * y axis (1) or z axis (2); 0 keeps the axes.  Exchanging axes leaves the
 * energy unchanged, so one network serves every axis. */
int dn_net_gather(dn_volume *vol, const int32_t *blocks_dev, int64_t n, int32_t perm, float *tiles_dev);

/* Workspace bytes of dn_net_forward (training 0) or dn_net_loss_grad
 * (training 1) on n tiles (0 for bad arguments). */
size_t dn_net_bytes(int64_t n_tiles, int32_t training);

/* Forward pass: out_dev float [n][10][10][10] (the residual r).
 * workspace_dev: device memory of dn_net_bytes(n, 0) bytes, 256-byte
 * aligned (else DN_E_CAPACITY / DN_E_INVALID). */
int dn_net_forward(const float *tiles_dev, int64_t n, const float *params_dev, float *out_dev,
                   void *workspace_dev, size_t workspace_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * forward pass of dn_net_forward with no workspace argument.  Its scratch
 * is a static device array inside the library (one per GPU, about 3.4 MB,
 * held until the process ends), so it takes at most DN_NET_STATIC_TILES
 * tiles per call (else DN_E_CAPACITY) and calls that overlap on one GPU
 * race (they share that array).  Same arguments and result as
 * dn_net_forward; enqueue only. */
#define DN_NET_STATIC_TILES 32
int dn_net_forward_static(const float *tiles_dev, int64_t n, const float *params_dev, float *out_dev,
                          void *hip_stream);

/* Masked mean-squared loss on the centre 8^3 and its gradient: the
 * prediction is f + r (kind 0, a primal residual) or r (kind 1, a dual
 * component); targets_dev, mask_dev float [n][512] in the tile's centre
 * order (mask 0/1); grad_dev float [8241] (overwritten).  *loss_host
 * receives the loss (synchronises).  workspace_dev: dn_net_bytes(n, 1)
 * bytes. */
int dn_net_loss_grad(const float *tiles_dev, int64_t n, const float *params_dev,
                     const float *targets_dev, const float *mask_dev, int32_t kind, float *grad_dev,
                     void *workspace_dev, size_t workspace_bytes, double *loss_host, void *hip_stream);

/* One Adam step on n float32 parameters (m, v: moments, step >= 1). */
int dn_net_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev, int64_t n,
                float lr, float beta1, float beta2, float eps, int32_t step, void *hip_stream);

/* Warm start of the whole volume (u0_dev float [n_blocks][512], p0_dev
 * float [3][n_blocks][512]):
 *  DN_WARM_PRIMAL: u0 = clamp(f + r, -1, 1) on Omega (0 elsewhere); p0
 *    (may be NULL) = projection of grad(u0) / delta onto the unit ball.
 *  DN_WARM_DUAL: the network runs once per axis a on tiles whose x axis is
 *    the volume's axis a and its output is taken as the dual component p_a
 *    (kept where m_a = 1); p0 is projected onto the unit ball and u0 = f on
 *    Omega.  delta is unused.
 * workspace_dev: device memory of dn_warm_start_bytes(number of blocks)
 * bytes, 256-byte aligned.  Enqueue only. */
#define DN_WARM_PRIMAL 0
#define DN_WARM_DUAL 1
size_t dn_warm_start_bytes(int64_t n_blocks);
int dn_net_warm_start(dn_volume *vol, const float *params_dev, int32_t mode, double delta,
                      float *u0_dev, float *p0_dev, void *workspace_dev, size_t workspace_bytes);

#ifdef __cplusplus
}
#endif
#endif /* DENSER_H */
