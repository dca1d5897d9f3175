/*
 * FP64 CPU oracle for sparse TSDF fusion and the Omega-masked TV
 * primal-dual regulariser of "DENSER Cities" (Tanner, Pinies, Paz, Newman).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header, table or helper with
 * the HIP library.
 *
 * Every floating-point value is double.  Build with -O2 -ffp-contract=off so
 * each discrete decision (block keys, pixel choice, truncation test) follows
 * IEEE double arithmetic in the written order.
 *
 * Parity status of each function is stated in its comment; every function
 * here is pinned by a CPU test against closed forms, invariants, brute force
 * or a library routine (see tests/test_oracle_pins.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_E_CAPACITY (-2)
#define BLK 8
#define NVOX 512

/* Linear voxel index inside a block: x fastest (x + 8y + 64z). */
static inline int lin(int x, int y, int z) { return x + BLK * y + BLK * BLK * z; }

/* floor division by 8 that is correct for negative integers */
static inline int32_t fdiv8(int32_t g) { return (g >= 0) ? g / 8 : -((-g + 7) / 8); }

/* ---------------------------------------------------------------------
 * Pixel validity (a reading: the paper does not say how invalid depth is
 * marked).  A depth is usable iff finite and in (0, max_depth].
 * ------------------------------------------------------------------- */
static inline int depth_valid(float d, double max_depth)
{
    return isfinite(d) && d > 0.0f && (double)d <= max_depth;
}

/* ---------------------------------------------------------------------
 * Block allocation, Section III-A: a whole block is allocated as soon as
 * a surface is observed somewhere inside it.
 * Reading: a pixel with depth d observes the band z in [d - mu, d + mu]
 * along its ray; every block that segment passes through is allocated.
 * The segment is walked with the Amanatides-Woo grid traversal over the
 * block grid (edge 8 s).  Ties between axes step x before y before z, and
 * only axes that still have steps left towards the end block are stepped.
 *
 * Emits (with repeats) every visited block key, up to max_out triples, and
 * returns the total number visited.
 * ------------------------------------------------------------------- */
int64_t or_candidates(const float *depth, int32_t W, int32_t H, const double *K4,
                      const double *T, double s, double mu, double max_depth,
                      int32_t *out, int64_t max_out)
{
    const double fx = K4[0], fy = K4[1], cx = K4[2], cy = K4[3];
    const double bs = 8.0 * s;
    int64_t n = 0;
    for (int32_t py = 0; py < H; ++py) {
        for (int32_t px = 0; px < W; ++px) {
            float d = depth[(int64_t)py * W + px];
            if (!depth_valid(d, max_depth)) continue;
            double rx = ((double)px - cx) / fx;
            double ry = ((double)py - cy) / fy;
            double z0 = (double)d - mu;
            if (z0 < 1e-3) z0 = 1e-3;
            double z1 = (double)d + mu;
            double a[3], b[3];
            for (int i = 0; i < 3; ++i) {
                /* camera point z*r, r = (rx, ry, 1); world = R * pc + t */
                double pa = ((T[4 * i + 0] * (z0 * rx) + T[4 * i + 1] * (z0 * ry)) + T[4 * i + 2] * z0) + T[4 * i + 3];
                double pb = ((T[4 * i + 0] * (z1 * rx) + T[4 * i + 1] * (z1 * ry)) + T[4 * i + 2] * z1) + T[4 * i + 3];
                a[i] = pa / bs;
                b[i] = pb / bs;
            }
            int skip = 0;
            for (int i = 0; i < 3; ++i)
                if (!(fabs(a[i]) < 1e6 && fabs(b[i]) < 1e6)) skip = 1;
            if (skip) continue;
            int64_t k[3], left[3];
            int step[3];
            double tmax[3], tdel[3];
            for (int i = 0; i < 3; ++i) {
                k[i] = (int64_t)floor(a[i]);
                int64_t e = (int64_t)floor(b[i]);
                double dir = b[i] - a[i];
                if (e > k[i]) {
                    step[i] = 1; left[i] = e - k[i];
                    tmax[i] = ((double)(k[i] + 1) - a[i]) / dir;
                    tdel[i] = 1.0 / dir;
                } else if (e < k[i]) {
                    step[i] = -1; left[i] = k[i] - e;
                    tmax[i] = ((double)k[i] - a[i]) / dir;
                    tdel[i] = -1.0 / dir;
                } else {
                    step[i] = 0; left[i] = 0; tmax[i] = 0.0; tdel[i] = 0.0;
                }
            }
            for (;;) {
                if (n < max_out) {
                    out[3 * n + 0] = (int32_t)k[0];
                    out[3 * n + 1] = (int32_t)k[1];
                    out[3 * n + 2] = (int32_t)k[2];
                }
                ++n;
                int c = -1;
                for (int i = 0; i < 3; ++i) {
                    if (left[i] == 0) continue;
                    if (c < 0 || tmax[i] < tmax[c]) c = i;
                }
                if (c < 0) break;
                k[c] += step[c];
                tmax[c] += tdel[c];
                left[c] -= 1;
            }
        }
    }
    return n;
}

/* ---------------------------------------------------------------------
 * Laser range data, Section III-A: the projective update extends to laser
 * sensors by updating only the voxels along each ray from the sensor to mu
 * behind the observed surface.  Readings: a return is a point p in the
 * sensor frame (T maps sensor to world); its range is r = |p|, valid iff
 * finite, r > 0 and r <= max_depth; the ray direction is p / r.  Points at
 * range rho along the ray are computed like the depth path's camera points,
 * world_i = ((T_i0 (rho d_x) + T_i1 (rho d_y)) + T_i2 (rho d_z)) + T_i3.
 *   Allocation: the blocks the band segment rho in [max(r - mu, 1e-3),
 *     r + mu] passes through (the depth path's rule), by the same traversal.
 *   Fusion: the voxel-grid traversal of rho in [0, r + mu]; a visited voxel
 *     of an allocated block with centre c gets eta = r - (c - o) . D (o the
 *     sensor origin, D the world direction) and, if eta >= -mu, the
 *     observation psi = min(1, eta / mu).  All observations of one scan are
 *     applied together: with k of them and S their sum (double, in ray
 *     order), f <- (w f + S) / (w + k), w <- w + k.
 * ------------------------------------------------------------------- */
typedef void (*cell_fn)(int64_t x, int64_t y, int64_t z, void *ctx);

/* Amanatides-Woo traversal of the segment a -> b on the unit grid, ties
 * x before y before z, only axes with steps left stepped (the traversal of
 * or_candidates).  Returns the number of cells. */
static int64_t walk_segment(const double a[3], const double b[3], cell_fn fn, void *ctx)
{
    for (int i = 0; i < 3; ++i)
        if (!(fabs(a[i]) < 1e9 && fabs(b[i]) < 1e9)) return 0;
    int64_t k[3], left[3];
    int step[3];
    double tmax[3], tdel[3];
    for (int i = 0; i < 3; ++i) {
        k[i] = (int64_t)floor(a[i]);
        int64_t e = (int64_t)floor(b[i]);
        double dir = b[i] - a[i];
        if (e > k[i]) {
            step[i] = 1; left[i] = e - k[i];
            tmax[i] = ((double)(k[i] + 1) - a[i]) / dir;
            tdel[i] = 1.0 / dir;
        } else if (e < k[i]) {
            step[i] = -1; left[i] = k[i] - e;
            tmax[i] = ((double)k[i] - a[i]) / dir;
            tdel[i] = -1.0 / dir;
        } else {
            step[i] = 0; left[i] = 0; tmax[i] = 0.0; tdel[i] = 0.0;
        }
    }
    int64_t n = 0;
    for (;;) {
        fn(k[0], k[1], k[2], ctx);
        ++n;
        int c = -1;
        for (int i = 0; i < 3; ++i) {
            if (left[i] == 0) continue;
            if (c < 0 || tmax[i] < tmax[c]) c = i;
        }
        if (c < 0) break;
        k[c] += step[c];
        tmax[c] += tdel[c];
        left[c] -= 1;
    }
    return n;
}

/* range and unit direction of a return; 0 if invalid */
static int laser_ray(const float *p, double max_depth, double *r, double d[3])
{
    if (!(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]))) return 0;
    double x = p[0], y = p[1], z = p[2];
    double rr = sqrt((x * x + y * y) + z * z);
    if (!(rr > 0.0 && rr <= max_depth)) return 0;
    *r = rr;
    d[0] = x / rr; d[1] = y / rr; d[2] = z / rr;
    return 1;
}

static void ray_point(const double *T, const double d[3], double rho, double out[3])
{
    for (int i = 0; i < 3; ++i)
        out[i] = ((T[4 * i + 0] * (rho * d[0]) + T[4 * i + 1] * (rho * d[1])) + T[4 * i + 2] * (rho * d[2])) + T[4 * i + 3];
}

typedef struct { int32_t *out; int64_t n, max_out; } cand_ctx;

static void cand_cell(int64_t x, int64_t y, int64_t z, void *vc)
{
    cand_ctx *c = (cand_ctx *)vc;
    if (c->n < c->max_out) {
        c->out[3 * c->n + 0] = (int32_t)x;
        c->out[3 * c->n + 1] = (int32_t)y;
        c->out[3 * c->n + 2] = (int32_t)z;
    }
    c->n++;
}

int64_t or_candidates_laser(const float *pts, int64_t n, const double *T, double s, double mu, double max_depth,
                            int32_t *out, int64_t max_out)
{
    cand_ctx c = {out, 0, max_out};
    const double bs = 8.0 * s;
    for (int64_t i = 0; i < n; ++i) {
        double r, d[3], pa[3], pb[3], a[3], b[3];
        if (!laser_ray(pts + 3 * i, max_depth, &r, d)) continue;
        double r0 = r - mu;
        if (r0 < 1e-3) r0 = 1e-3;
        ray_point(T, d, r0, pa);
        ray_point(T, d, r + mu, pb);
        for (int k = 0; k < 3; ++k) { a[k] = pa[k] / bs; b[k] = pb[k] / bs; }
        walk_segment(a, b, cand_cell, &c);
    }
    return c.n;
}

typedef struct {
    const int32_t *slots; int32_t cap, tail;
    double s, mu, r, o[3], D[3];
    double *sum; int64_t *cnt;
} fuse_ctx;

int32_t or_hash_find(const int32_t *slots, int32_t cap, int32_t tail, int32_t x, int32_t y, int32_t z);

static void fuse_cell(int64_t x, int64_t y, int64_t z, void *vc)
{
    fuse_ctx *c = (fuse_ctx *)vc;
    int32_t bx = fdiv8((int32_t)x), by = fdiv8((int32_t)y), bz = fdiv8((int32_t)z);
    int32_t id = or_hash_find(c->slots, c->cap, c->tail, bx, by, bz);
    if (id < 0) return;
    double rho = 0.0;
    double g[3] = {(double)x, (double)y, (double)z};
    for (int i = 0; i < 3; ++i) rho += ((g[i] + 0.5) * c->s - c->o[i]) * c->D[i];
    double eta = c->r - rho;
    if (eta < -c->mu) return;
    double psi = eta / c->mu;
    if (psi > 1.0) psi = 1.0;
    int64_t v = (int64_t)id * NVOX + lin((int)(x - 8 * (int64_t)bx), (int)(y - 8 * (int64_t)by), (int)(z - 8 * (int64_t)bz));
    c->sum[v] += psi;
    c->cnt[v] += 1;
}

void or_fuse_laser(const int32_t *slots, int32_t cap, int32_t tail, int64_t nb, double *f, double *w,
                   const float *pts, int64_t n, const double *T, double s, double mu, double max_depth)
{
    int64_t nv = nb * NVOX;
    double *sum = (double *)calloc((size_t)(nv > 0 ? nv : 1), sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)(nv > 0 ? nv : 1), sizeof(int64_t));
    fuse_ctx c;
    c.slots = slots; c.cap = cap; c.tail = tail; c.s = s; c.mu = mu; c.sum = sum; c.cnt = cnt;
    for (int i = 0; i < 3; ++i) {
        c.o[i] = T[4 * i + 3];
    }
    for (int64_t i = 0; i < n; ++i) {
        double r, d[3], pa[3], pb[3], a[3], b[3];
        if (!laser_ray(pts + 3 * i, max_depth, &r, d)) continue;
        c.r = r;
        for (int k = 0; k < 3; ++k) c.D[k] = (T[4 * k + 0] * d[0] + T[4 * k + 1] * d[1]) + T[4 * k + 2] * d[2];
        ray_point(T, d, 0.0, pa);
        ray_point(T, d, r + mu, pb);
        for (int k = 0; k < 3; ++k) { a[k] = pa[k] / s; b[k] = pb[k] / s; }
        walk_segment(a, b, fuse_cell, &c);
    }
    for (int64_t v = 0; v < nv; ++v) {
        if (cnt[v] == 0) continue;
        double wn = w[v] + (double)cnt[v];
        f[v] = (w[v] * f[v] + sum[v]) / wn;
        w[v] = wn;
    }
    free(sum);
    free(cnt);
}

/* ---------------------------------------------------------------------
 * Spatial hash (the paper cites Teschner et al. and Niessner et al. for
 * the hashing voxel grid without giving a function).  Reading: the
 * Teschner primes XOR-ed over the two's-complement coordinates, masked to
 * a power-of-two bucket count, with linear probing that never wraps (a tail
 * of extra slots follows the last bucket).
 * ------------------------------------------------------------------- */
uint32_t or_hash_home(int32_t x, int32_t y, int32_t z, uint32_t cap)
{
    uint32_t h = ((uint32_t)x * 73856093u) ^ ((uint32_t)y * 19349669u) ^ ((uint32_t)z * 83492791u);
    return h & (cap - 1u);
}

typedef struct { uint32_t home; int32_t x, y, z, id; } or_entry;

static int cmp_entry(const void *pa, const void *pb)
{
    const or_entry *a = (const or_entry *)pa, *b = (const or_entry *)pb;
    if (a->home != b->home) return a->home < b->home ? -1 : 1;
    if (a->x != b->x) return a->x < b->x ? -1 : 1;
    if (a->y != b->y) return a->y < b->y ? -1 : 1;
    if (a->z != b->z) return a->z < b->z ? -1 : 1;
    return 0;
}

/* Build the table by inserting the keys one after another in ascending
 * (home, x, y, z) order with plain linear probing.  Slot layout:
 * int32 {x, y, z, id}, id = -1 for an empty slot.  Returns OR_E_CAPACITY if
 * a key would fall past the last slot. */
int32_t or_hash_build(const int32_t *coords, int64_t n, int32_t cap, int32_t tail, int32_t *slots)
{
    int64_t nslot = (int64_t)cap + tail;
    for (int64_t i = 0; i < nslot; ++i) {
        slots[4 * i + 0] = 0; slots[4 * i + 1] = 0; slots[4 * i + 2] = 0; slots[4 * i + 3] = -1;
    }
    or_entry *e = (or_entry *)malloc(sizeof(or_entry) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        e[i].x = coords[3 * i]; e[i].y = coords[3 * i + 1]; e[i].z = coords[3 * i + 2];
        e[i].id = (int32_t)i;
        e[i].home = or_hash_home(e[i].x, e[i].y, e[i].z, (uint32_t)cap);
    }
    qsort(e, (size_t)n, sizeof(or_entry), cmp_entry);
    int32_t rc = OR_OK;
    for (int64_t i = 0; i < n; ++i) {
        int64_t pos = e[i].home;
        while (pos < nslot && slots[4 * pos + 3] >= 0) ++pos;
        if (pos >= nslot) { rc = OR_E_CAPACITY; break; }
        slots[4 * pos + 0] = e[i].x; slots[4 * pos + 1] = e[i].y;
        slots[4 * pos + 2] = e[i].z; slots[4 * pos + 3] = e[i].id;
    }
    free(e);
    return rc;
}

int32_t or_hash_find(const int32_t *slots, int32_t cap, int32_t tail, int32_t x, int32_t y, int32_t z)
{
    int64_t nslot = (int64_t)cap + tail;
    for (int64_t pos = or_hash_home(x, y, z, (uint32_t)cap); pos < nslot; ++pos) {
        const int32_t *sl = slots + 4 * pos;
        if (sl[3] < 0) return -1;
        if (sl[0] == x && sl[1] == y && sl[2] == z) return sl[3];
    }
    return -1;
}

/* 27-entry neighbourhood of every block: entry (dz+1)*9 + (dy+1)*3 + (dx+1)
 * holds the pool id of block + (dx, dy, dz), or -1 if it is not allocated.
 * The centre entry is the block itself. */
void or_nbr(const int32_t *coords, int64_t n, const int32_t *slots, int32_t cap, int32_t tail, int32_t *nbr)
{
    for (int64_t b = 0; b < n; ++b)
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx)
                    nbr[27 * b + (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] =
                        or_hash_find(slots, cap, tail, coords[3 * b] + dx, coords[3 * b + 1] + dy, coords[3 * b + 2] + dz);
}

/* ---------------------------------------------------------------------
 * Projective TSDF fusion, Section III-A, Eq. (1), for every voxel of every
 * listed block and one depth map.
 *   p_c = T_gc^-1 p_g  (T_gc camera->world, row-major 4x4: p_c = R^T (p_g - t))
 *   nearest pixel of the projection; if it lies in the map and is valid:
 *   eta = d - z_c; if eta >= -mu: w += 1, f = (psi + w_old f) / w,
 *   psi = min(1, eta / mu)   (reading: u_TSDF is the KinectFusion
 *   truncation normalised to [-1, 1]; the paper cites KinectFusion for the
 *   update and leaves u_TSDF undefined).
 * Voxel centre (g + 0.5) s, pixel centres at integer coordinates, nearest
 * pixel = floor(X + 0.5); voxels at or behind the camera plane are skipped.
 * ------------------------------------------------------------------- */
void or_fuse(const int32_t *coords, int64_t nb, double *f, double *w, const float *depth,
             int32_t W, int32_t H, const double *K4, const double *T, double s, double mu,
             double max_depth, int32_t nthreads)
{
    const double fx = K4[0], fy = K4[1], cx = K4[2], cy = K4[3];
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t b = 0; b < nb; ++b) {
        for (int v = 0; v < NVOX; ++v) {
            int l[3] = {v % 8, (v / 8) % 8, v / 64};
            double d3[3];
            for (int i = 0; i < 3; ++i) {
                double pg = ((double)(8 * coords[3 * b + i] + l[i]) + 0.5) * s;
                d3[i] = pg - T[4 * i + 3];
            }
            double xc = (T[0] * d3[0] + T[4] * d3[1]) + T[8] * d3[2];
            double yc = (T[1] * d3[0] + T[5] * d3[1]) + T[9] * d3[2];
            double zc = (T[2] * d3[0] + T[6] * d3[1]) + T[10] * d3[2];
            if (!(zc > 0.0)) continue;
            double X = fx * (xc / zc) + cx;
            double Y = fy * (yc / zc) + cy;
            double vx = X + 0.5, vy = Y + 0.5;
            if (!(vx >= 0.0 && vx < (double)W && vy >= 0.0 && vy < (double)H)) continue;
            int32_t px = (int32_t)floor(vx), py = (int32_t)floor(vy);
            float d = depth[(int64_t)py * W + px];
            if (!depth_valid(d, max_depth)) continue;
            double eta = (double)d - zc;
            if (eta < -mu) continue;
            double psi = eta / mu;
            if (psi > 1.0) psi = 1.0;
            int64_t idx = b * NVOX + v;
            double wo = w[idx];
            double wn = wo + 1.0;
            f[idx] = (psi + wo * f[idx]) / wn;
            w[idx] = wn;
        }
    }
}

/* ---------------------------------------------------------------------
 * Voxel addressing across block faces through the 27-neighbourhood.
 * (lx, ly, lz) in [-1, 8]; returns the global voxel index or -1 when the
 * voxel lies in a block that is not allocated.
 * ------------------------------------------------------------------- */
static inline int64_t vox_at(const int32_t *nbr, int64_t b, int lx, int ly, int lz)
{
    int dx = lx < 0 ? -1 : (lx > 7 ? 1 : 0);
    int dy = ly < 0 ? -1 : (ly > 7 ? 1 : 0);
    int dz = lz < 0 ? -1 : (lz > 7 ? 1 : 0);
    int32_t id = nbr[27 * b + (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
    if (id < 0) return -1;
    return (int64_t)id * NVOX + lin(lx - 8 * dx, ly - 8 * dy, lz - 8 * dz);
}

/* Omega, Section III-B: a voxel is in Omega iff its block is allocated and
 * it has been observed (w > 0).  Unallocated blocks are in Omega-bar. */
static inline int in_omega(const double *w, int64_t idx) { return idx >= 0 && w[idx] > 0.0; }

static const int EX[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

/* Masked forward-difference gradient, Eq. (3): component a is
 * u(g + e_a) - u(g) if both voxels are in Omega, else 0.  Block faces are
 * not grid ends: the difference crosses into the neighbour block when that
 * block is allocated and the voxel there is in Omega. */
static void grad_at(const int32_t *nbr, const double *w, const double *u, int64_t b, int v, double g[3])
{
    int l[3] = {v % 8, (v / 8) % 8, v / 64};
    int64_t i0 = b * NVOX + v;
    for (int a = 0; a < 3; ++a) {
        int64_t i1 = vox_at(nbr, b, l[0] + EX[a][0], l[1] + EX[a][1], l[2] + EX[a][2]);
        g[a] = (in_omega(w, i0) && in_omega(w, i1)) ? (u[i1] - u[i0]) : 0.0;
    }
}

/* Masked divergence, Eq. (4), taken as the negative adjoint of grad_at
 * (the paper defines it as the dual of the new gradient; its listed cases
 * overlap, and this reading reproduces each of them):
 *   div p(g) = sum_a [ m_a(g) p_a(g) - m_a(g - e_a) p_a(g - e_a) ],
 *   m_a(g) = [g in Omega][g + e_a in Omega].  Axes summed x, y, z. */
static double div_at(const int32_t *nbr, const double *w, const double *p, int64_t nvox, int64_t b, int v)
{
    int l[3] = {v % 8, (v / 8) % 8, v / 64};
    int64_t i0 = b * NVOX + v;
    double acc = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double *pa = p + (int64_t)a * nvox;
        int64_t ip = vox_at(nbr, b, l[0] + EX[a][0], l[1] + EX[a][1], l[2] + EX[a][2]);
        int64_t im = vox_at(nbr, b, l[0] - EX[a][0], l[1] - EX[a][1], l[2] - EX[a][2]);
        double fwd = (in_omega(w, i0) && in_omega(w, ip)) ? pa[i0] : 0.0;
        double bwd = (in_omega(w, im) && in_omega(w, i0)) ? pa[im] : 0.0;
        acc += fwd - bwd;
    }
    return acc;
}

/* exported single-voxel operators, for the adjoint and other pins */
void or_grad(const int32_t *nbr, int64_t nb, const double *w, const double *u, double *g_out /*[3][nb*512]*/)
{
    int64_t nvox = nb * NVOX;
    for (int64_t b = 0; b < nb; ++b)
        for (int v = 0; v < NVOX; ++v) {
            double g[3];
            grad_at(nbr, w, u, b, v, g);
            for (int a = 0; a < 3; ++a) g_out[a * nvox + b * NVOX + v] = g[a];
        }
}

void or_div(const int32_t *nbr, int64_t nb, const double *w, const double *p, double *d_out)
{
    int64_t nvox = nb * NVOX;
    for (int64_t b = 0; b < nb; ++b)
        for (int v = 0; v < NVOX; ++v) d_out[b * NVOX + v] = div_at(nbr, w, p, nvox, b, v);
}

/* ---------------------------------------------------------------------
 * Chambolle-Pock iteration, Section III-C, Eqs. (7)-(9), N iterations:
 *   dual:    p~ = p + sigma grad(ubar);  p = p~ / max(1, |p~|_2)   (Eq. 7)
 *   primal:  u~ = u + tau div p                                       (Eq. 8)
 *            u' = (u~ + tau lambda w f) / (1 + tau lambda w) on Omega,
 *            u' = u on Omega-bar (the regulariser acts only on Omega)
 *   relax:   ubar = u' + theta (u' - u)                               (Eq. 9)
 * Readings: Eq. (8) prints u - tau div p, which with div = -grad^T
 * diverges; the standard method (the paper's reference [Chambolle & Pock
 * 2011]) ascends in the dual and descends with -grad^T p = +div p.
 * Eq. (9) prints u + theta(u - ubar), which oscillates; the standard
 * extrapolation u_k + theta (u_k - u_{k-1}) is used.
 * p is stored as three planes [3][nb*512].  The state (u, ubar, p) is
 * updated in place so a split run resumes exactly.
 * ------------------------------------------------------------------- */
void or_cp(const int32_t *nbr, int64_t nb, const double *f, const double *w, double *u,
           double *ubar, double *p, int32_t iters, double lambda, double tau, double sigma,
           double theta, int32_t nthreads)
{
    int64_t nvox = nb * NVOX;
    int nt = nthreads > 0 ? nthreads : 1;
    for (int32_t it = 0; it < iters; ++it) {
        /* dual ascent + projection, every voxel reads the previous ubar */
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t b = 0; b < nb; ++b)
            for (int v = 0; v < NVOX; ++v) {
                double g[3], pt[3];
                grad_at(nbr, w, ubar, b, v, g);
                int64_t i0 = b * NVOX + v;
                for (int a = 0; a < 3; ++a) pt[a] = p[a * nvox + i0] + sigma * g[a];
                double nrm = sqrt((pt[0] * pt[0] + pt[1] * pt[1]) + pt[2] * pt[2]);
                double den = nrm > 1.0 ? nrm : 1.0;
                for (int a = 0; a < 3; ++a) p[a * nvox + i0] = pt[a] / den;
            }
        /* primal proximal step and relaxation, reads the new p */
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t b = 0; b < nb; ++b)
            for (int v = 0; v < NVOX; ++v) {
                int64_t i0 = b * NVOX + v;
                double uo = u[i0], un = uo;
                if (in_omega(w, i0)) {
                    double ut = uo + tau * div_at(nbr, w, p, nvox, b, v);
                    double tlw = tau * lambda * w[i0];
                    un = (ut + tlw * f[i0]) / (1.0 + tlw);
                }
                ubar[i0] = un + theta * (un - uo);
                u[i0] = un;
            }
    }
}

/* ---------------------------------------------------------------------
 * Accelerated variant (the paper's reference [Chambolle & Pock 2011], the
 * algorithm for a uniformly convex primal term): the data term
 * (lambda/2) w (u - f)^2 is uniformly convex with modulus gamma = lambda
 * min_Omega w, which allows step sizes that adapt every iteration:
 *   theta_n = 1 / sqrt(1 + 2 gamma tau_n),
 *   tau_{n+1} = theta_n tau_n,  sigma_{n+1} = sigma_n / theta_n,
 * with the dual and primal steps of or_cp using sigma_n, tau_n and the
 * relaxation using theta_n.  state[0..1] = (tau_n, sigma_n) on entry and
 * on exit, so a split run resumes exactly.
 * ------------------------------------------------------------------- */
void or_cp_accel(const int32_t *nbr, int64_t nb, const double *f, const double *w, double *u,
                 double *ubar, double *p, int32_t iters, double lambda, double gamma, double *state,
                 int32_t nthreads)
{
    for (int32_t it = 0; it < iters; ++it) {
        double tau = state[0], sigma = state[1];
        double theta = 1.0 / sqrt(1.0 + 2.0 * gamma * tau);
        or_cp(nbr, nb, f, w, u, ubar, p, 1, lambda, tau, sigma, theta, nthreads);
        state[0] = theta * tau;
        state[1] = sigma / theta;
    }
}

/* ---------------------------------------------------------------------
 * Primal and dual energies, Eq. (2) and Eqs. (5)-(6).
 * Reading: Eq. (2) prints lambda |f - u|^2 without the weight, but the
 * update of Eq. (8) is the proximal map of (lambda/2) w (u - f)^2; the
 * energy that matches the iteration is used:
 *   E(u) = sum_Omega |grad u|_2 + (lambda/2) w (u - f)^2
 *   D(p) = sum_Omega -f div p - (div p)^2 / (2 lambda w)
 * (D is the minimum over u of the Lagrangian -<u, div p> + data term.)
 * Sums: per block in voxel order, then blocks in pool order.
 * out[0] = E, out[1] = D.
 * ------------------------------------------------------------------- */
void or_energy(const int32_t *nbr, int64_t nb, const double *f, const double *w, const double *u,
               const double *p, double lambda, double *out, int32_t nthreads)
{
    int64_t nvox = nb * NVOX;
    double *pe = (double *)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
    double *pd = (double *)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t b = 0; b < nb; ++b) {
        double se = 0.0, sd = 0.0;
        for (int v = 0; v < NVOX; ++v) {
            int64_t i0 = b * NVOX + v;
            if (!in_omega(w, i0)) continue;
            double g[3];
            grad_at(nbr, w, u, b, v, g);
            double r = u[i0] - f[i0];
            se += sqrt((g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]) + 0.5 * lambda * w[i0] * r * r;
            double dv = div_at(nbr, w, p, nvox, b, v);
            sd += -f[i0] * dv - dv * dv / (2.0 * lambda * w[i0]);
        }
        pe[b] = se;
        pd[b] = sd;
    }
    double E = 0.0, D = 0.0;
    for (int64_t b = 0; b < nb; ++b) { E += pe[b]; D += pd[b]; }
    out[0] = E;
    out[1] = D;
    free(pe);
    free(pd);
}

/* ---------------------------------------------------------------------
 * TV-L1 variant of the same framework (the paper names the L1 norm as the
 * prior of its regulariser, Section III-B; this variant also takes the
 * data term in L1):
 *   E(u) = sum_Omega |grad u|_2 + lambda w |u - f|,   u in [-1, 1]
 * The box is the range of a truncated signed distance; with f in [-1, 1]
 * it does not change the minimiser (truncating u to [min f, max f] lowers
 * neither term).  The iteration is or_cp's with the proximal map of
 * tau lambda w |u - f| + box in place of the quadratic one: a soft
 * threshold of u~ - f by tau lambda w, then the clamp to [-1, 1] (for a
 * one-dimensional convex term plus an interval, the proximal map is the
 * interval projection of the term's proximal map).
 * ------------------------------------------------------------------- */
static double shrink(double x, double t) { return x > t ? x - t : (x < -t ? x + t : 0.0); }
static double clamp1(double x) { return x < -1.0 ? -1.0 : (x > 1.0 ? 1.0 : x); }

void or_cp_l1(const int32_t *nbr, int64_t nb, const double *f, const double *w, double *u,
              double *ubar, double *p, int32_t iters, double lambda, double tau, double sigma,
              double theta, int32_t nthreads)
{
    int64_t nvox = nb * NVOX;
    int nt = nthreads > 0 ? nthreads : 1;
    for (int32_t it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t b = 0; b < nb; ++b)
            for (int v = 0; v < NVOX; ++v) {
                double g[3], pt[3];
                grad_at(nbr, w, ubar, b, v, g);
                int64_t i0 = b * NVOX + v;
                for (int a = 0; a < 3; ++a) pt[a] = p[a * nvox + i0] + sigma * g[a];
                double nrm = sqrt((pt[0] * pt[0] + pt[1] * pt[1]) + pt[2] * pt[2]);
                double den = nrm > 1.0 ? nrm : 1.0;
                for (int a = 0; a < 3; ++a) p[a * nvox + i0] = pt[a] / den;
            }
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int64_t b = 0; b < nb; ++b)
            for (int v = 0; v < NVOX; ++v) {
                int64_t i0 = b * NVOX + v;
                double uo = u[i0], un = uo;
                if (in_omega(w, i0)) {
                    double ut = uo + tau * div_at(nbr, w, p, nvox, b, v);
                    un = clamp1(f[i0] + shrink(ut - f[i0], tau * lambda * w[i0]));
                }
                ubar[i0] = un + theta * (un - uo);
                u[i0] = un;
            }
    }
}

/* Energies of the TV-L1 variant.  The dual is the minimum over u in the box
 * of the Lagrangian -<u, div p> + lambda sum w |u - f|; per voxel the
 * minimum of that piecewise linear function of u over [-1, 1] lies at -1,
 * f or 1:
 *   D(p) = sum_Omega min(-f d, -d + lambda w |1 - f|, d + lambda w |1 + f|),
 * d = div p.  out[0] = E, out[1] = D. */
void or_energy_l1(const int32_t *nbr, int64_t nb, const double *f, const double *w, const double *u,
                  const double *p, double lambda, double *out, int32_t nthreads)
{
    int64_t nvox = nb * NVOX;
    double *pe = (double *)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
    double *pd = (double *)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t b = 0; b < nb; ++b) {
        double se = 0.0, sd = 0.0;
        for (int v = 0; v < NVOX; ++v) {
            int64_t i0 = b * NVOX + v;
            if (!in_omega(w, i0)) continue;
            double g[3];
            grad_at(nbr, w, u, b, v, g);
            se += sqrt((g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]) + lambda * w[i0] * fabs(u[i0] - f[i0]);
            double d = div_at(nbr, w, p, nvox, b, v);
            double lw = lambda * w[i0];
            double c0 = -f[i0] * d, c1 = -d + lw * fabs(1.0 - f[i0]), c2 = d + lw * fabs(1.0 + f[i0]);
            double m = c0 < c1 ? c0 : c1;
            sd += m < c2 ? m : c2;
        }
        pe[b] = se;
        pd[b] = sd;
    }
    double E = 0.0, D = 0.0;
    for (int64_t b = 0; b < nb; ++b) { E += pe[b]; D += pd[b]; }
    out[0] = E;
    out[1] = D;
    free(pe);
    free(pd);
}

/* ---------------------------------------------------------------------
 * Surface extraction (Section II: the zero-crossing level set of the TSDF).
 * For every voxel g and axis a with m_a(g) = 1 and a sign change between
 * u(g) and u(g + e_a) (sign = u < 0), the crossing point
 *   c(g) + t s e_a,  t = u(g) / (u(g) - u(g + e_a)),  c(g) = (g + 0.5) s
 * Order: pool id, voxel index, axis.  Writes up to max_out points and
 * returns the total number.
 * ------------------------------------------------------------------- */
int64_t or_extract(const int32_t *coords, const int32_t *nbr, int64_t nb, const double *w,
                   const double *u, double s, double *pts, int64_t max_out)
{
    int64_t n = 0;
    for (int64_t b = 0; b < nb; ++b)
        for (int v = 0; v < NVOX; ++v) {
            int l[3] = {v % 8, (v / 8) % 8, v / 64};
            int64_t i0 = b * NVOX + v;
            if (!in_omega(w, i0)) continue;
            for (int a = 0; a < 3; ++a) {
                int64_t i1 = vox_at(nbr, b, l[0] + EX[a][0], l[1] + EX[a][1], l[2] + EX[a][2]);
                if (!in_omega(w, i1)) continue;
                if ((u[i0] < 0.0) == (u[i1] < 0.0)) continue;
                double t = u[i0] / (u[i0] - u[i1]);
                if (n < max_out) {
                    for (int i = 0; i < 3; ++i) {
                        double c = ((double)(8 * coords[3 * b + i] + l[i]) + 0.5) * s;
                        pts[3 * n + i] = c + (i == a ? t * s : 0.0);
                    }
                }
                ++n;
            }
        }
    return n;
}

/* ---------------------------------------------------------------------
 * Triangle mesh of the zero level set (Section II: the surface is the
 * zero-crossing isosurface of the TSDF; the paper reports its area in
 * Tables III and IV).  Reading: only cubes whose eight corner voxels are
 * all observed (in Omega) are meshed.  Each cube (voxel g and g + {0,1}^3,
 * corner k = x + 2y + 4z) is split into six tetrahedra along its main
 * diagonal, one per axis order (a0, a1, a2):
 *   corners 0, e_a0, e_a0 + e_a1, 7,
 * in the order (0,1,2) (0,2,1) (1,0,2) (1,2,0) (2,0,1) (2,1,0); neighbouring
 * cubes split their shared faces alike, so the mesh has no cracks.  In a
 * tetrahedron with vertices q = 0..3 and signs u < 0:
 *   one vertex alone on its side: one triangle on the edges from it to the
 *     other three, in increasing q;
 *   two and two (negative a < b, positive c < d): the triangles
 *     (ac, ad, bd) and (ac, bd, bc).
 * An edge point is P_i + t (P_j - P_i), t = u_i / (u_i - u_j), taken from
 * the lower corner i (smaller k) so every cube computes a shared edge's
 * point identically; corner positions are (g + offset + 0.5) s.  A triangle
 * (A, B, C) is turned to (A, C, B) when its normal (B - A) x (C - A) points
 * against r = n_neg sum(positive corner offsets) - n_pos sum(negative
 * corner offsets), so normals point to u > 0.  Order: pool id, voxel index,
 * tetrahedron, triangle.  Writes up to max_out triangles (9 values each),
 * returns the total number, and the sum of the triangle areas (in that
 * order) in *area.
 * ------------------------------------------------------------------- */
static const int TET_AXES[6][2] = {{0, 1}, {0, 2}, {1, 0}, {1, 2}, {2, 0}, {2, 1}};

static void mesh_edge(const double P[8][3], const double uc[8], int ki, int kj, double out[3])
{
    if (ki > kj) { int x = ki; ki = kj; kj = x; }
    double t = uc[ki] / (uc[ki] - uc[kj]);
    for (int c = 0; c < 3; ++c) out[c] = P[ki][c] + t * (P[kj][c] - P[ki][c]);
}

static void mesh_tri(const double P[8][3], const double uc[8], const int kk[4], int e0a, int e0b, int e1a,
                     int e1b, int e2a, int e2b, const double r[3], double *tris, int64_t *n, int64_t max_out,
                     double *area)
{
    double A[3], B[3], C[3];
    mesh_edge(P, uc, kk[e0a], kk[e0b], A);
    mesh_edge(P, uc, kk[e1a], kk[e1b], B);
    mesh_edge(P, uc, kk[e2a], kk[e2b], C);
    double ab[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double ac[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    double nx = ab[1] * ac[2] - ab[2] * ac[1];
    double ny = ab[2] * ac[0] - ab[0] * ac[2];
    double nz = ab[0] * ac[1] - ab[1] * ac[0];
    int flip = (nx * r[0] + ny * r[1]) + nz * r[2] < 0.0;
    *area += 0.5 * sqrt((nx * nx + ny * ny) + nz * nz);
    if (*n < max_out) {
        double *o = tris + 9 * (*n);
        for (int c = 0; c < 3; ++c) {
            o[c] = A[c];
            o[3 + c] = flip ? C[c] : B[c];
            o[6 + c] = flip ? B[c] : C[c];
        }
    }
    ++(*n);
}

int64_t or_mesh(const int32_t *coords, const int32_t *nbr, int64_t nb, const double *w, const double *u,
                double s, double *tris, int64_t max_out, double *area)
{
    int64_t n = 0;
    double ar = 0.0;
    for (int64_t b = 0; b < nb; ++b)
        for (int v = 0; v < NVOX; ++v) {
            int l[3] = {v % 8, (v / 8) % 8, v / 64};
            double uc[8], P[8][3];
            int ok = 1;
            for (int k = 0; k < 8 && ok; ++k) {
                int o[3] = {k & 1, (k >> 1) & 1, (k >> 2) & 1};
                int64_t idx = vox_at(nbr, b, l[0] + o[0], l[1] + o[1], l[2] + o[2]);
                if (!in_omega(w, idx)) { ok = 0; break; }
                uc[k] = u[idx];
                for (int c = 0; c < 3; ++c) P[k][c] = ((double)(8 * coords[3 * b + c] + l[c] + o[c]) + 0.5) * s;
            }
            if (!ok) continue;
            for (int tt = 0; tt < 6; ++tt) {
                int a0 = TET_AXES[tt][0], a1 = TET_AXES[tt][1];
                int kk[4] = {0, 1 << a0, (1 << a0) | (1 << a1), 7};
                int neg[4], nneg = 0;
                for (int q = 0; q < 4; ++q) { neg[q] = uc[kk[q]] < 0.0; nneg += neg[q]; }
                if (nneg == 0 || nneg == 4) continue;
                double r[3] = {0.0, 0.0, 0.0};
                for (int q = 0; q < 4; ++q)
                    for (int c = 0; c < 3; ++c) {
                        double oc = (double)((kk[q] >> c) & 1);
                        r[c] += neg[q] ? -(double)(4 - nneg) * oc : (double)nneg * oc;
                    }
                if (nneg == 1 || nneg == 3) {
                    int odd = -1, j[3], m = 0;
                    for (int q = 0; q < 4; ++q)
                        if (neg[q] == (nneg == 1)) odd = q;
                    for (int q = 0; q < 4; ++q)
                        if (q != odd) j[m++] = q;
                    mesh_tri(P, uc, kk, odd, j[0], odd, j[1], odd, j[2], r, tris, &n, max_out, &ar);
                } else {
                    int ng[2], ps[2], mn = 0, mp = 0;
                    for (int q = 0; q < 4; ++q) {
                        if (neg[q]) ng[mn++] = q;
                        else ps[mp++] = q;
                    }
                    int a = ng[0], bb = ng[1], c = ps[0], d = ps[1];
                    mesh_tri(P, uc, kk, a, c, a, d, bb, d, r, tris, &n, max_out, &ar);
                    mesh_tri(P, uc, kk, a, c, bb, d, bb, c, r, tris, &n, max_out, &ar);
                }
            }
        }
    *area = ar;
    return n;
}

/* ---------------------------------------------------------------------
 * Learned warm start: a 3-layer 3x3x3 convolutional network on a 10^3 tile
 * (an 8^3 block plus a one-voxel halo) with two input channels (fused f and
 * the normalised weight), 16 hidden channels with ReLU, one output channel.
 * "same" zero padding inside the tile.  Everything here is plain loops in
 * double.  Parameter layout (8241 values, this order):
 *   W1[16][2][27] b1[16] W2[16][16][27] b2[16] W3[1][16][27] b3[1]
 * with tap index (dz*3 + dy)*3 + dx.
 * ------------------------------------------------------------------- */
#define T10 10
#define T3 1000
#define HID 16

static void conv_same(const double *x, int cin, const double *Wt, const double *bias, int cout,
                      double *y)
{
    for (int co = 0; co < cout; ++co)
        for (int z = 0; z < T10; ++z)
            for (int yy = 0; yy < T10; ++yy)
                for (int xx = 0; xx < T10; ++xx) {
                    double acc = bias[co];
                    for (int ci = 0; ci < cin; ++ci)
                        for (int dz = 0; dz < 3; ++dz)
                            for (int dy = 0; dy < 3; ++dy)
                                for (int dx = 0; dx < 3; ++dx) {
                                    int zz = z + dz - 1, y2 = yy + dy - 1, x2 = xx + dx - 1;
                                    if (zz < 0 || zz >= T10 || y2 < 0 || y2 >= T10 || x2 < 0 || x2 >= T10) continue;
                                    acc += Wt[(co * cin + ci) * 27 + (dz * 3 + dy) * 3 + dx] *
                                           x[ci * T3 + (zz * T10 + y2) * T10 + x2];
                                }
                    y[co * T3 + (z * T10 + yy) * T10 + xx] = acc;
                }
}

/* Round to the nearest bfloat16 value (ties to even), through float32 as
 * the device sees its float32 inputs, weights and accumulators.  Used only
 * to take the ReLU decisions in the network's own operand precision. */
static double to_bf16(double v)
{
    float f = (float)v;
    uint32_t bits;
    memcpy(&bits, &f, sizeof bits);
    if ((bits & 0x7f800000u) != 0x7f800000u) {
        uint32_t lsb = (bits >> 16) & 1u;
        bits = bits + 0x7fffu + lsb;
    }
    bits &= 0xffff0000u;
    memcpy(&f, &bits, sizeof f);
    return (double)f;
}

/* Forward pass for a batch of tiles.  tiles: [B][2][10][10][10];
 * out: [B][10][10][10] residual r (the caller crops the centre 8^3).
 * If acts is not NULL it receives the pre-activations of layers 1 and 2,
 * [B][2][16][1000], and gates (same shape) the values whose sign opens
 * each ReLU, for the backward pass.
 * gate 0: a ReLU is open where its float64 pre-activation is > 0.
 * gate 1: the network is specified to run with bfloat16 operands, and an
 *   open/closed ReLU is a discrete decision, so it is taken in that
 *   precision: a second forward pass whose inputs, weights and layer inputs
 *   are rounded to bfloat16 (float64 sums, biases unrounded) decides which
 *   ReLUs are open; the values themselves stay float64.  The layer-1
 *   weights, to which the output is most sensitive, are the pair
 *   bf16(W) + bf16(W - bf16(W)) in that pass (the network's layer-1
 *   operands).
 * gate 2: the output is that second pass itself, carried through layer 3
 *   (its input and weights rounded to bfloat16 too): the network evaluated
 *   with every operand in its own precision and float64 sums, so that it
 *   differs from a float32-accumulating evaluation only by the order and
 *   precision of the sums. */
void or_net_forward(const double *tiles, int64_t B, const double *params, double *out, double *acts,
                    double *gates, int32_t gate)
{
    const double *W1 = params, *b1 = W1 + HID * 2 * 27, *W2 = b1 + HID, *b2 = W2 + HID * HID * 27,
                 *W3 = b2 + HID, *b3 = W3 + HID * 27;
    const int nw1 = HID * 2 * 27, nw2 = HID * HID * 27;
    double *h1 = (double *)malloc(sizeof(double) * HID * T3);
    double *h2 = (double *)malloc(sizeof(double) * HID * T3);
    double *g1 = (double *)malloc(sizeof(double) * HID * T3);
    double *g2 = (double *)malloc(sizeof(double) * HID * T3);
    double *xr = (double *)malloc(sizeof(double) * 2 * T3);
    double *W1r = (double *)malloc(sizeof(double) * nw1);
    double *W2r = (double *)malloc(sizeof(double) * nw2);
    double W3r[HID * 27];
    for (int i = 0; i < nw1; ++i) W1r[i] = to_bf16(W1[i]) + to_bf16(W1[i] - to_bf16(W1[i]));
    for (int i = 0; i < nw2; ++i) W2r[i] = to_bf16(W2[i]);
    for (int i = 0; i < HID * 27; ++i) W3r[i] = to_bf16(W3[i]);
    for (int64_t bi = 0; bi < B; ++bi) {
        const double *x = tiles + bi * 2 * T3;
        conv_same(x, 2, W1, b1, HID, h1);
        if (gate) {
            for (int i = 0; i < 2 * T3; ++i) xr[i] = to_bf16(x[i]);
            conv_same(xr, 2, W1r, b1, HID, g1);
        } else {
            memcpy(g1, h1, sizeof(double) * HID * T3);
        }
        if (acts) {
            memcpy(acts + (bi * 2 + 0) * HID * T3, h1, sizeof(double) * HID * T3);
            memcpy(gates + (bi * 2 + 0) * HID * T3, g1, sizeof(double) * HID * T3);
        }
        for (int i = 0; i < HID * T3; ++i) {
            h1[i] = g1[i] > 0.0 ? h1[i] : 0.0;
            g1[i] = g1[i] > 0.0 ? to_bf16(g1[i]) : 0.0;
        }
        conv_same(h1, HID, W2, b2, HID, h2);
        if (gate) conv_same(g1, HID, W2r, b2, HID, g2);
        else memcpy(g2, h2, sizeof(double) * HID * T3);
        if (acts) {
            memcpy(acts + (bi * 2 + 1) * HID * T3, h2, sizeof(double) * HID * T3);
            memcpy(gates + (bi * 2 + 1) * HID * T3, g2, sizeof(double) * HID * T3);
        }
        if (gate == 2) {
            for (int i = 0; i < HID * T3; ++i) g2[i] = g2[i] > 0.0 ? to_bf16(g2[i]) : 0.0;
            conv_same(g2, HID, W3r, b3, 1, out + bi * T3);
            continue;
        }
        for (int i = 0; i < HID * T3; ++i) h2[i] = g2[i] > 0.0 ? h2[i] : 0.0;
        conv_same(h2, HID, W3, b3, 1, out + bi * T3);
    }
    free(h1); free(h2); free(g1); free(g2); free(xr); free(W1r); free(W2r);
}

/* Variance of rounding a value to bfloat16 (round to nearest): the error
 * is spread evenly over one spacing of the bfloat16 grid at v, whose
 * 8-bit significand gives the spacing 2^(e - 8) for |v| in [2^(e-1), 2^e). */
static double bf16_round_var(double v)
{
    if (v == 0.0) return 0.0;
    int e;
    frexp(v, &e);
    double ulp = ldexp(1.0, e - 8);
    return ulp * ulp / 12.0;
}

/* Standard deviation, element by element over the 10^3 output of each
 * tile, of the difference between the float64 network (gate 0) and an
 * evaluation that rounds the inputs, the layer-2 and layer-3 weights and
 * the inputs of layers 2 and 3 to bfloat16, modelling every rounding error
 * as an independent zero-mean variable of variance bf16_round_var of the
 * rounded value and propagating the variances through the layers (a
 * convolution with the squared weights; a closed ReLU, taken from the
 * float64 pre-activation, passes nothing).  The layer-1 weight pair
 * (relative error 2^-16), the biases (not rounded) and float32 sums (unit
 * roundoff 2^-24) are below this model's resolution and left out:
 *   V1 = (W1^2) * var(x)
 *   V_{l+1} = (W_{l+1}^2) * (open_l (V_l + var(h_l))) + (var(W_{l+1})) * h_l^2
 * The L2 norm of the returned field is the expected L2 norm of the
 * difference. */
void or_net_error_rms(const double *tiles, int64_t B, const double *params, double *out)
{
    const double *W1 = params, *b1 = W1 + HID * 2 * 27, *W2 = b1 + HID, *b2 = W2 + HID * HID * 27,
                 *W3 = b2 + HID;
    const int nw1 = HID * 2 * 27, nw2 = HID * HID * 27;
    double *sW1 = (double *)malloc(sizeof(double) * nw1), *sW2 = (double *)malloc(sizeof(double) * nw2);
    double *vW2 = (double *)malloc(sizeof(double) * nw2);
    double sW3[HID * 27], vW3[HID * 27], zero[HID];
    for (int i = 0; i < nw1; ++i) sW1[i] = W1[i] * W1[i];
    for (int i = 0; i < nw2; ++i) { sW2[i] = W2[i] * W2[i]; vW2[i] = bf16_round_var(W2[i]); }
    for (int i = 0; i < HID * 27; ++i) { sW3[i] = W3[i] * W3[i]; vW3[i] = bf16_round_var(W3[i]); }
    for (int i = 0; i < HID; ++i) zero[i] = 0.0;
    double *h = (double *)malloc(sizeof(double) * HID * T3), *hn = (double *)malloc(sizeof(double) * HID * T3);
    double *V = (double *)malloc(sizeof(double) * HID * T3), *h2sq = (double *)malloc(sizeof(double) * HID * T3);
    double *c = (double *)malloc(sizeof(double) * HID * T3), *a = (double *)malloc(sizeof(double) * HID * T3);
    double *vx = (double *)malloc(sizeof(double) * 2 * T3);
    for (int64_t bi = 0; bi < B; ++bi) {
        const double *x = tiles + bi * 2 * T3;
        for (int i = 0; i < 2 * T3; ++i) vx[i] = bf16_round_var((double)(float)x[i]);
        conv_same(x, 2, W1, b1, HID, h);
        conv_same(vx, 2, sW1, zero, HID, V);
        for (int layer = 2; layer <= 3; ++layer) {
            const int cout = layer == 2 ? HID : 1;
            for (int i = 0; i < HID * T3; ++i) {
                const int open = h[i] > 0.0;
                h[i] = open ? h[i] : 0.0;
                V[i] = open ? V[i] + bf16_round_var(h[i]) : 0.0;
                h2sq[i] = h[i] * h[i];
            }
            conv_same(V, HID, layer == 2 ? sW2 : sW3, zero, cout, c);
            conv_same(h2sq, HID, layer == 2 ? vW2 : vW3, zero, cout, a);
            if (layer == 2) {
                conv_same(h, HID, W2, b2, HID, hn);
                memcpy(h, hn, sizeof(double) * HID * T3);
                for (int i = 0; i < HID * T3; ++i) V[i] = c[i] + a[i];
            } else {
                for (int i = 0; i < T3; ++i) out[bi * T3 + i] = sqrt(c[i] + a[i]);
            }
        }
    }
    free(sW1); free(sW2); free(vW2); free(h); free(hn); free(V); free(h2sq); free(c); free(a); free(vx);
}

/* Gradient of a same-padded convolution y = conv(x, W) + b given dy:
 * accumulates dW, db and (if dx != NULL) writes dx. */
static void conv_same_backward(const double *x, int cin, const double *Wt, int cout, const double *dy,
                               double *dW, double *db, double *dx)
{
    if (dx) memset(dx, 0, sizeof(double) * (size_t)cin * T3);
    for (int co = 0; co < cout; ++co)
        for (int z = 0; z < T10; ++z)
            for (int yy = 0; yy < T10; ++yy)
                for (int xx = 0; xx < T10; ++xx) {
                    double g = dy[co * T3 + (z * T10 + yy) * T10 + xx];
                    db[co] += g;
                    for (int ci = 0; ci < cin; ++ci)
                        for (int dz = 0; dz < 3; ++dz)
                            for (int dyy = 0; dyy < 3; ++dyy)
                                for (int dxx = 0; dxx < 3; ++dxx) {
                                    int zz = z + dz - 1, y2 = yy + dyy - 1, x2 = xx + dxx - 1;
                                    if (zz < 0 || zz >= T10 || y2 < 0 || y2 >= T10 || x2 < 0 || x2 >= T10) continue;
                                    int widx = (co * cin + ci) * 27 + (dz * 3 + dyy) * 3 + dxx;
                                    int xidx = ci * T3 + (zz * T10 + y2) * T10 + x2;
                                    dW[widx] += g * x[xidx];
                                    if (dx) dx[xidx] += g * Wt[widx];
                                }
                }
}

/* Masked mean-squared loss on the centre 8^3 of each tile and its gradient
 * with respect to all parameters:
 *   pred = f_centre + r_centre (kind 0: the network is a primal residual) or
 *   pred = r_centre (kind 1: the network predicts a dual component),
 *   L = sum_mask (pred - target)^2 / max(1, n_mask)
 * targets, mask: [B][512] (block voxel order of the tile's centre); mask is
 * 0/1.  grad: [8241], overwritten.  Returns L. */
double or_net_loss_grad(const double *tiles, int64_t B, const double *params, const double *targets,
                        const double *mask, double *grad, int32_t kind, int32_t gate)
{
    const double *W1 = params, *W2 = params + HID * 2 * 27 + HID, *W3 = W2 + HID * HID * 27 + HID;
    double *gW1 = grad, *gb1 = gW1 + HID * 2 * 27, *gW2 = gb1 + HID, *gb2 = gW2 + HID * HID * 27,
           *gW3 = gb2 + HID, *gb3 = gW3 + HID * 27;
    memset(grad, 0, sizeof(double) * 8241);
    double *acts = (double *)malloc(sizeof(double) * (size_t)B * 2 * HID * T3);
    double *gates = (double *)malloc(sizeof(double) * (size_t)B * 2 * HID * T3);
    double *out = (double *)malloc(sizeof(double) * (size_t)B * T3);
    or_net_forward(tiles, B, params, out, acts, gates, gate);
    double nmask = 0.0;
    for (int64_t i = 0; i < B * 512; ++i) nmask += mask[i];
    double norm = nmask > 1.0 ? nmask : 1.0;
    double loss = 0.0;
    double *d3 = (double *)malloc(sizeof(double) * T3);
    double *h = (double *)malloc(sizeof(double) * HID * T3);
    double *dh = (double *)malloc(sizeof(double) * HID * T3);
    double *dh1 = (double *)malloc(sizeof(double) * HID * T3);
    for (int64_t bi = 0; bi < B; ++bi) {
        memset(d3, 0, sizeof(double) * T3);
        for (int v = 0; v < 512; ++v) {
            int x = v % 8 + 1, y = (v / 8) % 8 + 1, z = v / 64 + 1;
            int t = (z * T10 + y) * T10 + x;
            double m = mask[bi * 512 + v];
            if (m == 0.0) continue;
            double pred = (kind == 0 ? tiles[bi * 2 * T3 + t] : 0.0) + out[bi * T3 + t];
            double e = pred - targets[bi * 512 + v];
            loss += e * e / norm;
            d3[t] = 2.0 * e / norm;
        }
        const double *a1 = acts + (bi * 2 + 0) * HID * T3, *a2 = acts + (bi * 2 + 1) * HID * T3;
        const double *o1 = gates + (bi * 2 + 0) * HID * T3, *o2 = gates + (bi * 2 + 1) * HID * T3;
        /* layer 3: input relu(a2), open where o2 > 0 */
        for (int i = 0; i < HID * T3; ++i) h[i] = o2[i] > 0.0 ? a2[i] : 0.0;
        conv_same_backward(h, HID, W3, 1, d3, gW3, gb3, dh);
        for (int i = 0; i < HID * T3; ++i) dh[i] = o2[i] > 0.0 ? dh[i] : 0.0;
        /* layer 2: input relu(a1), open where o1 > 0 */
        for (int i = 0; i < HID * T3; ++i) h[i] = o1[i] > 0.0 ? a1[i] : 0.0;
        conv_same_backward(h, HID, W2, HID, dh, gW2, gb2, dh1);
        for (int i = 0; i < HID * T3; ++i) dh1[i] = o1[i] > 0.0 ? dh1[i] : 0.0;
        /* layer 1: input tile */
        conv_same_backward(tiles + bi * 2 * T3, 2, W1, HID, dh1, gW1, gb1, NULL);
    }
    free(acts); free(gates); free(out); free(d3); free(h); free(dh); free(dh1);
    return loss;
}

/* Gather the network input tile of each listed block: channel 0 = f,
 * channel 1 = log(1 + w) / log(1 + 100), over the block and a one-voxel
 * halo; voxels of unallocated neighbours are 0 in both channels.
 * perm turns the volume so that one of its axes becomes the tile's x axis:
 * 0 none, 1 x and y exchanged, 2 x and z exchanged (the energy is
 * unchanged by exchanging axes, so one network serves every axis). */
void or_net_gather(const int32_t *nbr, const double *f, const double *w, const int32_t *blocks,
                   int64_t n, double *tiles, int32_t perm)
{
    const double wn = log(101.0);
    for (int64_t i = 0; i < n; ++i) {
        int64_t b = blocks[i];
        for (int z = 0; z < T10; ++z)
            for (int y = 0; y < T10; ++y)
                for (int x = 0; x < T10; ++x) {
                    int t = (z * T10 + y) * T10 + x;
                    int vx = x, vy = y, vz = z;
                    if (perm == 1) { vx = y; vy = x; }
                    if (perm == 2) { vx = z; vz = x; }
                    int64_t idx = vox_at(nbr, b, vx - 1, vy - 1, vz - 1);
                    double fv = 0.0, wv = 0.0;
                    if (idx >= 0) { fv = f[idx]; wv = log(1.0 + w[idx]) / wn; }
                    tiles[i * 2 * T3 + t] = fv;
                    tiles[i * 2 * T3 + T3 + t] = wv;
                }
    }
}
