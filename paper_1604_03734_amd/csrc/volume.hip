// Volume lifecycle, block allocation (grid traversal, dedupe, canonical
// hash), projective TSDF fusion and plain extraction for gfx950.
//
// Section III-A of the paper (hashing voxel grid, Eq. 1).  Discrete
// decisions (block keys, pixel choice, truncation test) are taken in
// float64 with contraction disabled, so they are reproducible bit for bit.
#include <cstring>  // rocprim needs memset declared before its headers
#include <rocprim/rocprim.hpp>

#include <cstdarg>
#include <algorithm>
#include <cmath>

#include "dn_internal.h"

namespace dn {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int read_back(dn_volume *v, const void *dev, size_t bytes)
{
    if (bytes > sizeof(v->host_stage)) { set_error("read-back too large"); return DN_E_INVALID; }
    DN_HIP(hipMemcpyAsync(v->host_stage, dev, bytes, hipMemcpyDeviceToHost, v->stream));
    DN_HIP(hipStreamSynchronize(v->stream));
    return DN_OK;
}

int volume_sync(dn_volume *v)
{
    DN_HIP(hipStreamSynchronize(v->stream));
    return DN_OK;
}

// ------------------------------------------------------------ block keys
constexpr int64_t kKeyOff = int64_t(1) << 20;   // 21 bits per axis

__host__ __device__ inline uint64_t pack_key(int32_t x, int32_t y, int32_t z)
{
    return (uint64_t(int64_t(x) + kKeyOff) << 42) | (uint64_t(int64_t(y) + kKeyOff) << 21) |
           uint64_t(int64_t(z) + kKeyOff);
}

__host__ __device__ inline void unpack_key(uint64_t k, int32_t &x, int32_t &y, int32_t &z)
{
    const uint64_t m = (uint64_t(1) << 21) - 1;
    x = int32_t(int64_t((k >> 42) & m) - kKeyOff);
    y = int32_t(int64_t((k >> 21) & m) - kKeyOff);
    z = int32_t(int64_t(k & m) - kKeyOff);
}

__device__ inline uint32_t bucket_of(int32_t x, int32_t y, int32_t z, uint32_t cap)
{
    uint32_t h = (uint32_t(x) * 73856093u) ^ (uint32_t(y) * 19349669u) ^ (uint32_t(z) * 83492791u);
    return h & (cap - 1u);
}

// Probe forward from the bucket until the key or an empty slot; the table
// never wraps, so the walk is bounded by the slot count.
__device__ inline int32_t hash_lookup(const int4 *slots, int64_t nslots, uint32_t cap, int32_t x,
                                      int32_t y, int32_t z)
{
    for (int64_t pos = bucket_of(x, y, z, cap); pos < nslots; ++pos) {
        int4 sl = slots[pos];
        if (sl.w < 0) return -1;
        if (sl.x == x && sl.y == y && sl.z == z) return sl.w;
    }
    return -1;
}

struct Geo {
    double fx, fy, cx, cy;
    double T[16];
    double s, mu, maxd;
    int32_t W, H;
};

__device__ inline bool depth_ok(float d, double maxd)
{
    return isfinite(d) && d > 0.0f && double(d) <= maxd;
}

// Amanatides-Woo traversal of a -> b on the unit grid (ties x before y
// before z, only axes with steps left towards the end cell); nothing is
// visited if an end point lies beyond `limit` cells.  Shared by the depth
// band, the laser band and the laser fusion walks.
template <class Emit>
__device__ int64_t walk_segment(const double a[3], const double b[3], double limit, Emit emit)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (!(fabs(a[i]) < limit && fabs(b[i]) < limit)) return 0;
    int64_t k[3], left[3];
    int step[3];
    double tmax[3], tdel[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        k[i] = int64_t(floor(a[i]));
        const int64_t e = int64_t(floor(b[i]));
        const double dir = b[i] - a[i];
        if (e > k[i]) {
            step[i] = 1; left[i] = e - k[i];
            tmax[i] = (double(k[i] + 1) - a[i]) / dir;
            tdel[i] = 1.0 / dir;
        } else if (e < k[i]) {
            step[i] = -1; left[i] = k[i] - e;
            tmax[i] = (double(k[i]) - a[i]) / dir;
            tdel[i] = -1.0 / dir;
        } else {
            step[i] = 0; left[i] = 0; tmax[i] = 0.0; tdel[i] = 0.0;
        }
    }
    int64_t n = 0;
    for (;;) {
        emit(n, k[0], k[1], k[2]);
        ++n;
        int c = -1;
#pragma unroll
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

// Grid traversal of one pixel's band [max(d - mu, 1e-3), d + mu] over the
// block grid (edge 8 s).  Emits the visited block keys through `emit` and
// returns how many were visited.
template <class Emit>
__device__ int dda_pixel(const Geo &g, int px, int py, float d, Emit emit)
{
    const double bs = 8.0 * g.s;
    double rx = (double(px) - g.cx) / g.fx;
    double ry = (double(py) - g.cy) / g.fy;
    double z0 = double(d) - g.mu;
    if (z0 < 1e-3) z0 = 1e-3;
    double z1 = double(d) + g.mu;
    double a[3], b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double pa = ((g.T[4 * i + 0] * (z0 * rx) + g.T[4 * i + 1] * (z0 * ry)) + g.T[4 * i + 2] * z0) + g.T[4 * i + 3];
        double pb = ((g.T[4 * i + 0] * (z1 * rx) + g.T[4 * i + 1] * (z1 * ry)) + g.T[4 * i + 2] * z1) + g.T[4 * i + 3];
        a[i] = pa / bs;
        b[i] = pb / bs;
    }
    return int(walk_segment(a, b, 1e6, [&](int64_t j, int64_t x, int64_t y, int64_t z) {
        emit(int(j), int32_t(x), int32_t(y), int32_t(z));
    }));
}

__global__ void k_dda_count(Geo g, const float *__restrict__ depth, int32_t *__restrict__ counts)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(g.W) * g.H) return;
    int px = int(i % g.W), py = int(i / g.W);
    float d = depth[i];
    int n = 0;
    if (depth_ok(d, g.maxd)) n = dda_pixel(g, px, py, d, [](int, int32_t, int32_t, int32_t) {});
    counts[i] = n;
}

__global__ void k_dda_emit(Geo g, const float *__restrict__ depth, const int32_t *__restrict__ offsets,
                           uint64_t *__restrict__ out, int64_t total)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(g.W) * g.H) return;
    int px = int(i % g.W), py = int(i / g.W);
    float d = depth[i];
    if (!depth_ok(d, g.maxd)) return;
    int64_t base = offsets[i];
    dda_pixel(g, px, py, d, [&](int j, int32_t x, int32_t y, int32_t z) {
        if (base + j < total) out[base + j] = pack_key(x, y, z);
    });
}

__global__ void k_pack_coords(const int32_t *__restrict__ c3, int64_t n, uint64_t *__restrict__ out)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = pack_key(c3[3 * i], c3[3 * i + 1], c3[3 * i + 2]);
}

// flag[i] = 1 if uniq[i] is not in the table (only i < *count is valid)
__global__ void k_flag_new(const uint64_t *__restrict__ uniq, const int64_t *__restrict__ count,
                           const int4 *__restrict__ slots, int64_t nslots, uint32_t cap,
                           uint8_t *__restrict__ flag, int64_t n_max)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_max) return;
    if (i >= *count) { flag[i] = 0; return; }
    int32_t x, y, z;
    unpack_key(uniq[i], x, y, z);
    flag[i] = hash_lookup(slots, nslots, cap, x, y, z) < 0 ? 1 : 0;
}

// flag[i] = 1 when raw candidate i (repeats allowed) is not in the table.
__global__ void k_flag_unknown(const uint64_t *__restrict__ cand, int64_t n, const int4 *__restrict__ slots,
                               int64_t nslots, uint32_t cap, uint8_t *__restrict__ flag)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t x, y, z;
    unpack_key(cand[i], x, y, z);
    flag[i] = hash_lookup(slots, nslots, cap, x, y, z) < 0 ? 1 : 0;
}

// Append the sorted new keys after the existing pool; clear their fields.
__global__ void k_append(const uint64_t *__restrict__ newk, int64_t n_new, int64_t nb_old,
                         int32_t *__restrict__ coords, uint64_t *__restrict__ keys)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_new) return;
    int32_t x, y, z;
    unpack_key(newk[i], x, y, z);
    int64_t b = nb_old + i;
    keys[b] = newk[i];
    coords[4 * b + 0] = x; coords[4 * b + 1] = y; coords[4 * b + 2] = z; coords[4 * b + 3] = 0;
}

// The per-voxel fields of blocks [first, first + count) in several arrays
// at once (the new blocks of an allocation: f, w, u, both ubar and both
// sets of dual planes), one launch instead of one per array.
struct FieldSet {
    float *a[16];
    int n;
};
__global__ void k_zero_fields(FieldSet fs, int64_t first, int64_t count)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count * kBlockVox) return;
    const int64_t off = first * kBlockVox + i;
    for (int k = 0; k < fs.n; ++k) fs.a[k][off] = 0.f;
}

__global__ void k_zero_blocks(float *__restrict__ a, int64_t first, int64_t count)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count * kBlockVox) a[first * kBlockVox + i] = 0.0f;
}

__global__ void k_iota(int32_t *__restrict__ a, int64_t n)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) a[i] = int32_t(i);
}

__global__ void k_bucket_of_keys(const uint64_t *__restrict__ keys, int64_t n, uint32_t cap,
                                 uint32_t *__restrict__ home)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t x, y, z;
    unpack_key(keys[i], x, y, z);
    home[i] = bucket_of(x, y, z, cap);
}

// d[i] = home_sorted[i] - i (as int64), scanned later with max
__global__ void k_home_minus_rank(const uint32_t *__restrict__ home, int64_t n, int64_t *__restrict__ d)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) d[i] = int64_t(home[i]) - i;
}

__global__ void k_zero_i32(int32_t *a) { *a = 0; }

__global__ void k_fill_empty(int4 *__restrict__ slots, int64_t n)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) slots[i] = make_int4(0, 0, 0, -1);
}

// Canonical slot of the i-th key in (bucket, key) order:
// pos = max_{j<=i}(home_j - j) + i  (sequential linear probing, unrolled)
__global__ void k_scatter_slots(const int64_t *__restrict__ runmax, const int32_t *__restrict__ ids,
                                const int32_t *__restrict__ coords, int64_t n, int64_t nslots,
                                int4 *__restrict__ slots, int32_t *__restrict__ overflow)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t pos = runmax[i] + i;
    if (pos >= nslots) { atomicOr(overflow, 1); return; }
    int32_t id = ids[i];
    slots[pos] = make_int4(coords[4 * id], coords[4 * id + 1], coords[4 * id + 2], id);
}

__global__ void k_nbr_table(const int32_t *__restrict__ coords, int64_t nb, const int4 *__restrict__ slots,
                            int64_t nslots, uint32_t cap, int32_t *__restrict__ nbr)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nb * kNbr) return;
    int64_t b = i / kNbr;
    int o = int(i % kNbr);
    int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
    nbr[i] = (o == kCentre) ? int32_t(b)
                            : hash_lookup(slots, nslots, cap, coords[4 * b] + dx,
                                          coords[4 * b + 1] + dy, coords[4 * b + 2] + dz);
}

static inline unsigned grid1(int64_t n, int bs = 256) { return unsigned((n + bs - 1) / bs); }

static int bits_for(uint64_t v)
{
    int b = 1;
    while (b < 64 && (v >> b)) ++b;
    return b;
}

InsertScratch carve_insert(Bump &b, int64_t n_cand, int64_t n_blocks)
{
    InsertScratch x;
    x.flags = b.take<uint8_t>(size_t(n_cand));
    x.newraw = b.take<uint64_t>(size_t(n_cand));
    x.sorted = b.take<uint64_t>(size_t(n_cand));
    x.newk = b.take<uint64_t>(size_t(n_cand));
    x.pos0 = b.take<int32_t>(size_t(n_cand));
    x.pos1 = b.take<int32_t>(size_t(n_cand));
    x.ksorted = b.take<uint64_t>(size_t(n_blocks));
    x.ids0 = b.take<int32_t>(size_t(n_blocks));
    x.ids1 = b.take<int32_t>(size_t(n_blocks));
    x.home = b.take<uint32_t>(size_t(n_blocks));
    x.home2 = b.take<uint32_t>(size_t(n_blocks));
    x.dm = b.take<int64_t>(size_t(n_blocks));
    x.runmax = b.take<int64_t>(size_t(n_blocks));
    x.tmp_bytes = std::max(std::max(tmp_sort(size_t(n_cand), 12), tmp_light(size_t(n_cand))),
                           std::max(tmp_sort(size_t(n_blocks), 12), tmp_light(size_t(n_blocks))));
    x.tmp = b.take<char>(x.tmp_bytes);
    return x;
}

// flags[i] = 1 where sorted[i] starts a run of equal keys
__global__ void k_run_heads(const uint64_t *__restrict__ sorted, int64_t n, uint8_t *__restrict__ flags)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = (i == 0 || sorted[i] != sorted[i - 1]) ? 1 : 0;
}

__global__ void k_gather_keys(const uint64_t *__restrict__ keys, const int32_t *__restrict__ pos, int64_t n,
                              uint64_t *__restrict__ out)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = keys[pos[i]];
}

// Insert a packed candidate list (device, n_cand entries, repeats allowed).
// Appends the keys not yet present in ascending order (keep_order: in the
// order of their first occurrence in the list), rebuilds hash +
// neighbours.  The raw list is first filtered against the table, so only
// candidates of new blocks are sorted (after the first frames of a sequence
// almost every candidate is a block that exists); the ascending list of all
// distinct candidates is built from the same raw list only when it is
// extracted (build_candidates).  All buffers come from the volume's scratch.
static int insert_packed(dn_volume *v, uint64_t *cand, int64_t n_cand, int32_t *n_new_out, bool keep_order = false)
{
    hipStream_t st = v->stream;
    if (n_new_out) *n_new_out = 0;
    v->cand_n = n_cand;
    if (n_cand == 0) return DN_OK;
    Bump bump(v->scratch, v->scratch_bytes);
    InsertScratch x = carve_insert(bump, n_cand, v->cap_blocks);
    if (!bump.fits()) { set_error("scratch too small for %lld candidates", (long long)n_cand); return DN_E_CAPACITY; }
    int64_t *d_nraw = v->misc;
    int64_t *d_nnew = d_nraw + 1;
    size_t tbytes;
    // 1) the candidates of blocks not in the table (repeats kept)
    const int4 *slots = reinterpret_cast<const int4 *>(v->hash[v->cur_hash]);
    hipLaunchKernelGGL(k_flag_unknown, dim3(grid1(n_cand)), dim3(256), 0, st, cand, n_cand, slots,
                       v->hash_slots, v->hash_cap, x.flags);
    DN_HIP(hipGetLastError());
    tbytes = x.tmp_bytes;
    DN_HIP(rocprim::select(x.tmp, tbytes, cand, x.flags, x.newraw, d_nraw, size_t(n_cand), st));
    int rc = read_back(v, d_nraw, sizeof(int64_t));
    if (rc) return rc;
    const int64_t n_raw = v->host_stage[0];
    if (n_raw == 0) return DN_OK;
    // 2) the distinct new keys, ascending (keep_order: in first-occurrence
    // order: a stable sort of (key, position), the first position of each
    // run of equal keys, those positions sorted, the keys gathered)
    if (!keep_order) {
        tbytes = x.tmp_bytes;
        DN_HIP(rocprim::radix_sort_keys(x.tmp, tbytes, x.newraw, x.sorted, size_t(n_raw), 0, 63, st));
        tbytes = x.tmp_bytes;
        DN_HIP(rocprim::unique(x.tmp, tbytes, x.sorted, x.newk, d_nnew, size_t(n_raw), rocprim::equal_to<uint64_t>(),
                               st));
    } else {
        hipLaunchKernelGGL(k_iota, dim3(grid1(n_raw)), dim3(256), 0, st, x.pos0, n_raw);
        DN_HIP(hipGetLastError());
        tbytes = x.tmp_bytes;
        DN_HIP(rocprim::radix_sort_pairs(x.tmp, tbytes, x.newraw, x.sorted, x.pos0, x.pos1, size_t(n_raw), 0, 63, st));
        hipLaunchKernelGGL(k_run_heads, dim3(grid1(n_raw)), dim3(256), 0, st, x.sorted, n_raw, x.flags);
        DN_HIP(hipGetLastError());
        tbytes = x.tmp_bytes;
        DN_HIP(rocprim::select(x.tmp, tbytes, x.pos1, x.flags, x.pos0, d_nnew, size_t(n_raw), st));
    }
    if ((rc = read_back(v, d_nnew, sizeof(int64_t)))) return rc;
    const int64_t n_new = v->host_stage[0];
    if (keep_order && n_new > 0) {
        tbytes = x.tmp_bytes;
        DN_HIP(rocprim::radix_sort_keys(x.tmp, tbytes, x.pos0, x.pos1, size_t(n_new), 0, bits_for(uint64_t(n_raw)),
                                        st));
        hipLaunchKernelGGL(k_gather_keys, dim3(grid1(n_new)), dim3(256), 0, st, x.newraw, x.pos1, n_new, x.newk);
        DN_HIP(hipGetLastError());
    }
    if (v->nb + n_new > v->cap_blocks) {
        set_error("block pool full: %lld + %lld new blocks > max_blocks %lld", (long long)v->nb,
                  (long long)n_new, (long long)v->cap_blocks);
        return DN_E_CAPACITY;
    }
    // 3) tentatively append (beyond nb; not committed until the hash fits)
    const int64_t nb_old = v->nb, nb_new = v->nb + n_new;
    hipLaunchKernelGGL(k_append, dim3(grid1(n_new)), dim3(256), 0, st, x.newk, n_new, nb_old, v->coords, v->keys);
    DN_HIP(hipGetLastError());
    // 4) canonical table: sort (key -> id), then stable sort by bucket
    hipLaunchKernelGGL(k_iota, dim3(grid1(nb_new)), dim3(256), 0, st, x.ids0, nb_new);
    DN_HIP(hipGetLastError());
    const int hbits = bits_for(v->hash_cap - 1);
    tbytes = x.tmp_bytes;
    DN_HIP(rocprim::radix_sort_pairs(x.tmp, tbytes, v->keys, x.ksorted, x.ids0, x.ids1, size_t(nb_new), 0, 63, st));
    hipLaunchKernelGGL(k_bucket_of_keys, dim3(grid1(nb_new)), dim3(256), 0, st, x.ksorted, nb_new, v->hash_cap, x.home);
    DN_HIP(hipGetLastError());
    tbytes = x.tmp_bytes;
    DN_HIP(rocprim::radix_sort_pairs(x.tmp, tbytes, x.home, x.home2, x.ids1, x.ids0, size_t(nb_new), 0, hbits, st));
    hipLaunchKernelGGL(k_home_minus_rank, dim3(grid1(nb_new)), dim3(256), 0, st, x.home2, nb_new, x.dm);
    DN_HIP(hipGetLastError());
    tbytes = x.tmp_bytes;
    DN_HIP(rocprim::inclusive_scan(x.tmp, tbytes, x.dm, x.runmax, size_t(nb_new), rocprim::maximum<int64_t>(), st));
    int other = 1 - v->cur_hash;
    int4 *dst = reinterpret_cast<int4 *>(v->hash[other]);
    int32_t *d_ovf = reinterpret_cast<int32_t *>(d_nraw + 2);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, st, d_ovf);
    hipLaunchKernelGGL(k_fill_empty, dim3(grid1(v->hash_slots)), dim3(256), 0, st, dst, v->hash_slots);
    DN_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scatter_slots, dim3(grid1(nb_new)), dim3(256), 0, st, x.runmax, x.ids0, v->coords, nb_new,
                       v->hash_slots, dst, d_ovf);
    DN_HIP(hipGetLastError());
    if ((rc = read_back(v, d_ovf, sizeof(int32_t)))) return rc;
    if (int32_t(v->host_stage[0] & 0xFFFFFFFF) != 0) {
        set_error("hash table full: %lld keys do not fit 2^%d buckets + %d tail slots", (long long)nb_new,
                  v->prm.hash_cap_log2, v->prm.hash_tail);
        return DN_E_CAPACITY;
    }
    // 5) commit: new table, zeroed fields of the new blocks, neighbours
    v->cur_hash = other;
    FieldSet fs{};
    float *fields[] = {v->f, v->w, v->u, v->ubar[0], v->ubar[1]};
    for (float *a : fields) fs.a[fs.n++] = a;
    for (int pp = 0; pp < 2; ++pp)
        for (int a = 0; a < 3; ++a) fs.a[fs.n++] = v->p[pp] + size_t(a) * v->cap_blocks * kBlockVox;
    hipLaunchKernelGGL(k_zero_fields, dim3(grid1(n_new * kBlockVox)), dim3(256), 0, st, fs, nb_old, n_new);
    DN_HIP(hipGetLastError());
    v->nb = nb_new;
    v->emask_nb = -1;
    v->state_storage = DN_F32;
    hipLaunchKernelGGL(k_nbr_table, dim3(grid1(nb_new * kNbr)), dim3(256), 0, st, v->coords, nb_new, dst,
                       v->hash_slots, v->hash_cap, v->nbr);
    DN_HIP(hipGetLastError());
    if (n_new_out) *n_new_out = int32_t(n_new);
    return DN_OK;
}

// ---------------------------------------------------------------- fusion
constexpr int kMiscFuseCount = 16;      // v->misc slot of the in-view block count
constexpr int64_t kFuseGrid = 4096;     // workgroups striding over the in-view list

// Eq. 1 for one voxel (k in 0..511, x fastest) of block b: project its
// centre, take the depth of the pixel it falls in, and average the
// truncated signed distance in with weight 1.  Voxels behind the camera,
// outside the image, with an invalid depth or more than mu behind the
// observed surface keep their values; free space in front of the surface
// is updated with the truncated value 1.
__device__ inline void fuse_voxel(const Geo &g, const float *__restrict__ depth, const int32_t *__restrict__ coords,
                                  int64_t b, int k, float *__restrict__ f, float *__restrict__ w)
{
    const int vx = k & 7, vy = (k >> 3) & 7, vz = (k >> 6) & 7;
    double d0 = (double(8 * coords[4 * b + 0] + vx) + 0.5) * g.s - g.T[3];
    double d1 = (double(8 * coords[4 * b + 1] + vy) + 0.5) * g.s - g.T[7];
    double d2 = (double(8 * coords[4 * b + 2] + vz) + 0.5) * g.s - g.T[11];
    double xc = (g.T[0] * d0 + g.T[4] * d1) + g.T[8] * d2;
    double yc = (g.T[1] * d0 + g.T[5] * d1) + g.T[9] * d2;
    double zc = (g.T[2] * d0 + g.T[6] * d1) + g.T[10] * d2;
    if (!(zc > 0.0)) return;
    double X = g.fx * (xc / zc) + g.cx;
    double Y = g.fy * (yc / zc) + g.cy;
    double px = X + 0.5, py = Y + 0.5;
    if (!(px >= 0.0 && px < double(g.W) && py >= 0.0 && py < double(g.H))) return;
    int ix = int(floor(px)), iy = int(floor(py));
    float d = depth[int64_t(iy) * g.W + ix];
    if (!depth_ok(d, g.maxd)) return;
    double eta = double(d) - zc;
    if (eta < -g.mu) return;
    double psi = eta / g.mu;
    if (psi > 1.0) psi = 1.0;
    const int64_t i = b * kBlockVox + k;
    float wo = w[i];
    float wn = wo + 1.0f;
    f[i] = (float(psi) + wo * f[i]) / wn;
    w[i] = wn;
}

// Visibility culling for fusion: can any voxel centre of the block pass
// the camera tests of fuse_voxel?  The centres span a box whose image in
// camera coordinates is a parallelepiped (the pose is affine), so depth
// ranges over the corners' depths; if all corners lie in front of the
// camera the box projects into the convex hull of the projected corners.
// Conservative: margins of 1e-6 m in depth and one pixel in the image
// absorb rounding differences from the per-voxel evaluation, and a box
// reaching behind the camera counts as visible.  A block is skipped only if
// every centre is behind the camera, beyond max_depth + mu (where no valid
// depth can put it within mu of a surface) or outside the image.
__device__ inline bool block_in_view(const Geo &g, const int32_t *c)
{
    double zmin = 1e300, zmax = -1e300, xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    double xs[8], ys[8], zs[8];
    for (int k = 0; k < 8; ++k) {
        double d0 = (double(8 * c[0] + ((k & 1) ? 7 : 0)) + 0.5) * g.s - g.T[3];
        double d1 = (double(8 * c[1] + ((k & 2) ? 7 : 0)) + 0.5) * g.s - g.T[7];
        double d2 = (double(8 * c[2] + ((k & 4) ? 7 : 0)) + 0.5) * g.s - g.T[11];
        xs[k] = (g.T[0] * d0 + g.T[4] * d1) + g.T[8] * d2;
        ys[k] = (g.T[1] * d0 + g.T[5] * d1) + g.T[9] * d2;
        zs[k] = (g.T[2] * d0 + g.T[6] * d1) + g.T[10] * d2;
        zmin = fmin(zmin, zs[k]);
        zmax = fmax(zmax, zs[k]);
    }
    const double eps = 1e-6;
    if (zmax <= -eps || zmin > g.maxd + g.mu + eps) return false;
    if (zmin <= eps) return true;
    for (int k = 0; k < 8; ++k) {
        double X = g.fx * (xs[k] / zs[k]) + g.cx + 0.5, Y = g.fy * (ys[k] / zs[k]) + g.cy + 0.5;
        xmin = fmin(xmin, X); xmax = fmax(xmax, X);
        ymin = fmin(ymin, Y); ymax = fmax(ymax, Y);
    }
    return xmax >= -1.0 && xmin < double(g.W) + 1.0 && ymax >= -1.0 && ymin < double(g.H) + 1.0;
}

// The blocks in view, appended to `list` (one atomic per wavefront; the
// order of the list varies, the fused values do not: every voxel is
// updated by one thread).
__global__ void k_cull(Geo g, const int32_t *__restrict__ coords, int64_t nb, int32_t *__restrict__ list,
                       int32_t *__restrict__ count)
{
    int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    bool vis = b < nb && block_in_view(g, coords + 4 * b);
    uint64_t m = __ballot(vis);
    if (m == 0) return;
    const int lane = __lane_id(), leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, leader);
    if (vis) list[base + __popcll(m & ((uint64_t(1) << lane) - 1))] = int32_t(b);
}

// Eq. 1 over the blocks in view: workgroups stride over the list (its
// length is read on the device, so the grid is sized from the pool).
__global__ __launch_bounds__(256) void k_fuse_list(Geo g, const float *__restrict__ depth,
                                                   const int32_t *__restrict__ coords,
                                                   const int32_t *__restrict__ list, const int32_t *__restrict__ count,
                                                   float *__restrict__ f, float *__restrict__ w)
{
    const int32_t n = *count;
    for (int32_t j = blockIdx.x; j < n; j += gridDim.x) {
        const int64_t b = list[j];
        fuse_voxel(g, depth, coords, b, threadIdx.x, f, w);
        fuse_voxel(g, depth, coords, b, threadIdx.x + 256, f, w);
    }
}

static int make_geo(const dn_volume *v, const dn_intrinsics *K, const double *T, Geo &g)
{
    DN_REQUIRE(K && T, "null intrinsics or pose");
    DN_REQUIRE(K->width > 0 && K->height > 0 && K->fx != 0.0 && K->fy != 0.0, "bad intrinsics");
    for (int i = 0; i < 16; ++i) DN_REQUIRE(std::isfinite(T[i]), "non-finite pose");
    g.fx = K->fx; g.fy = K->fy; g.cx = K->cx; g.cy = K->cy;
    for (int i = 0; i < 16; ++i) g.T[i] = T[i];
    g.s = v->prm.voxel_size; g.mu = v->prm.mu; g.maxd = v->prm.max_depth;
    g.W = K->width; g.H = K->height;
    return DN_OK;
}

// ------------------------------------------------------------------ laser
// Laser range data (Section III-A: the projective update extends to laser
// sensors by updating only the voxels along each ray from the sensor to mu
// behind the observed surface).  A return is a point p in the sensor frame
// (T: sensor -> world), range r = |p|, valid iff finite, 0 < r <= max_depth,
// direction d = p / r; the point at range rho is
// ((T_i0 (rho d_x) + T_i1 (rho d_y)) + T_i2 (rho d_z)) + T_i3.
//   Allocation: the blocks met by the band rho in [max(r - mu, 1e-3), r + mu].
//   Fusion: the voxels met by rho in [0, r + mu] in allocated blocks with
//   eta = r - (c - o) . D >= -mu give psi = min(1, eta / mu); one scan's
//   observations are applied together, f <- (w f + sum psi) / (w + k),
//   w <- w + k, the sum in float64 (a segmented reduction over the
//   observations sorted by voxel).
struct LGeo {
    double T[16];
    double s, mu, maxd;
};

__device__ inline bool laser_ray(const float *p, double maxd, double &r, double d[3])
{
    if (!(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]))) return false;
    const double x = p[0], y = p[1], z = p[2];
    const double rr = sqrt((x * x + y * y) + z * z);
    if (!(rr > 0.0 && rr <= maxd)) return false;
    r = rr;
    d[0] = x / rr; d[1] = y / rr; d[2] = z / rr;
    return true;
}

__device__ inline void ray_point(const double *T, const double d[3], double rho, double out[3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
        out[i] = ((T[4 * i + 0] * (rho * d[0]) + T[4 * i + 1] * (rho * d[1])) + T[4 * i + 2] * (rho * d[2])) +
                 T[4 * i + 3];
}

template <class Emit>
__device__ int64_t laser_band(const LGeo &g, const float *p, Emit emit)
{
    double r, d[3], pa[3], pb[3], a[3], b[3];
    if (!laser_ray(p, g.maxd, r, d)) return 0;
    double r0 = r - g.mu;
    if (r0 < 1e-3) r0 = 1e-3;
    ray_point(g.T, d, r0, pa);
    ray_point(g.T, d, r + g.mu, pb);
    const double bs = 8.0 * g.s;
#pragma unroll
    for (int i = 0; i < 3; ++i) { a[i] = pa[i] / bs; b[i] = pb[i] / bs; }
    return walk_segment(a, b, 1e9, emit);
}

__global__ void k_laser_cand_count(LGeo g, const float *__restrict__ pts, int64_t n, int32_t *__restrict__ counts)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    counts[i] = int32_t(laser_band(g, pts + 3 * i, [](int64_t, int64_t, int64_t, int64_t) {}));
}

__global__ void k_laser_cand_emit(LGeo g, const float *__restrict__ pts, int64_t n, const int32_t *__restrict__ offsets,
                                  uint64_t *__restrict__ out, int64_t total)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t base = offsets[i];
    laser_band(g, pts + 3 * i, [&](int64_t j, int64_t x, int64_t y, int64_t z) {
        if (base + j < total) out[base + j] = pack_key(int32_t(x), int32_t(y), int32_t(z));
    });
}

// The observations of one return: emit(j, voxel index, psi) for each visited
// voxel of an allocated block with eta >= -mu; returns their number.
template <class Emit>
__device__ int64_t laser_obs(const LGeo &g, const float *p, const int4 *slots, int64_t nslots, uint32_t cap,
                             Emit emit)
{
    double r, d[3], pa[3], pb[3], a[3], b[3], D[3];
    if (!laser_ray(p, g.maxd, r, d)) return 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) D[i] = (g.T[4 * i + 0] * d[0] + g.T[4 * i + 1] * d[1]) + g.T[4 * i + 2] * d[2];
    ray_point(g.T, d, 0.0, pa);
    ray_point(g.T, d, r + g.mu, pb);
#pragma unroll
    for (int i = 0; i < 3; ++i) { a[i] = pa[i] / g.s; b[i] = pb[i] / g.s; }
    int64_t m = 0;
    int64_t kb[3] = {INT64_MIN, 0, 0};
    int32_t id = -1;
    walk_segment(a, b, 1e9, [&](int64_t, int64_t x, int64_t y, int64_t z) {
        const int64_t bx = x >> 3, by = y >> 3, bz = z >> 3;   // floor division
        if (bx != kb[0] || by != kb[1] || bz != kb[2]) {
            kb[0] = bx; kb[1] = by; kb[2] = bz;
            id = hash_lookup(slots, nslots, cap, int32_t(bx), int32_t(by), int32_t(bz));
        }
        if (id < 0) return;
        const double gg[3] = {double(x), double(y), double(z)};
        double rho = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) rho += ((gg[i] + 0.5) * g.s - g.T[4 * i + 3]) * D[i];
        const double eta = r - rho;
        if (eta < -g.mu) return;
        double psi = eta / g.mu;
        if (psi > 1.0) psi = 1.0;
        const int64_t v = int64_t(id) * kBlockVox + ((x - 8 * bx) + 8 * (y - 8 * by) + 64 * (z - 8 * bz));
        emit(m, v, psi);
        ++m;
    });
    return m;
}

__global__ void k_laser_obs_count(LGeo g, const float *__restrict__ pts, int64_t n, const int4 *__restrict__ slots,
                                  int64_t nslots, uint32_t cap, int64_t *__restrict__ counts)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    counts[i] = laser_obs(g, pts + 3 * i, slots, nslots, cap, [](int64_t, int64_t, double) {});
}

__global__ void k_laser_obs_emit(LGeo g, const float *__restrict__ pts, int64_t n, const int4 *__restrict__ slots,
                                 int64_t nslots, uint32_t cap, const int64_t *__restrict__ offsets,
                                 uint32_t *__restrict__ keys, double *__restrict__ vals, int64_t total)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t base = offsets[i];
    laser_obs(g, pts + 3 * i, slots, nslots, cap, [&](int64_t j, int64_t v, double psi) {
        if (base + j < total) {
            keys[base + j] = uint32_t(v);
            vals[base + j] = psi;
        }
    });
}

// One scan's update of each observed voxel, from the per-voxel sums and
// counts of its observations (a segmented reduction of the sorted list).
__global__ void k_laser_apply(const uint32_t *__restrict__ uniq, const double *__restrict__ sums,
                              const uint32_t *__restrict__ counts, const uint32_t *__restrict__ nruns, int64_t m,
                              float *__restrict__ f, float *__restrict__ w)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m || i >= int64_t(*nruns)) return;
    const uint32_t v = uniq[i];
    const double w0 = w[v];
    const double wn = w0 + double(counts[i]);
    f[v] = float((w0 * double(f[v]) + sums[i]) / wn);
    w[v] = float(wn);
}

static int make_lgeo(const dn_volume *v, const double *T, LGeo &g)
{
    DN_REQUIRE(T, "null pose");
    for (int i = 0; i < 16; ++i) DN_REQUIRE(std::isfinite(T[i]), "non-finite pose");
    for (int i = 0; i < 16; ++i) g.T[i] = T[i];
    g.s = v->prm.voxel_size; g.mu = v->prm.mu; g.maxd = v->prm.max_depth;
    return DN_OK;
}

// Scratch of one laser fusion call: per-return counts and offsets, the
// observation lists (voxel key, psi) and their sorted copies, the per-voxel
// counts and the rocprim storage.
struct LaserScratch {
    int64_t *counts, *offs;
    uint32_t *k_in, *k_out, *counts32, *nruns;
    double *v_in, *v_out;
    void *tmp;
    size_t tmp_bytes;
};
static LaserScratch carve_laser(Bump &b, int64_t n, int64_t m)
{
    LaserScratch x;
    x.counts = b.take<int64_t>(size_t(n));
    x.offs = b.take<int64_t>(size_t(n) + 1);
    x.k_in = b.take<uint32_t>(size_t(m));
    x.k_out = b.take<uint32_t>(size_t(m));
    x.counts32 = b.take<uint32_t>(size_t(m));
    x.nruns = b.take<uint32_t>(1);
    x.v_in = b.take<double>(size_t(m));
    x.v_out = b.take<double>(size_t(m));
    x.tmp_bytes = std::max(std::max(tmp_light(size_t(n)), tmp_light(size_t(m))), tmp_sort(size_t(m), 12));
    x.tmp = b.take<char>(x.tmp_bytes);
    return x;
}

// Scratch of the band count of one frame (or scan) of n points.
struct FrameScratch {
    int32_t *counts, *offs;
    void *tmp;
    size_t tmp_bytes;
};
static FrameScratch carve_frame(Bump &b, int64_t n)
{
    FrameScratch x;
    x.counts = b.take<int32_t>(size_t(n));
    x.offs = b.take<int32_t>(size_t(n) + 2);
    x.tmp_bytes = tmp_light(size_t(n));
    x.tmp = b.take<char>(x.tmp_bytes);
    return x;
}

struct CandScratch {
    uint64_t *sorted, *uniq;
    void *tmp;
    size_t tmp_bytes;
};
static CandScratch carve_cand(Bump &b, int64_t n)
{
    CandScratch x;
    x.sorted = b.take<uint64_t>(size_t(n));
    x.uniq = b.take<uint64_t>(size_t(n));
    x.tmp_bytes = std::max(tmp_sort(size_t(n), 8), tmp_light(size_t(n)));
    x.tmp = b.take<char>(x.tmp_bytes);
    return x;
}

size_t candidates_scratch(int64_t n_cand)
{
    Bump b(nullptr, 0);
    carve_cand(b, n_cand);
    return b.off;
}

// The ascending distinct keys of the last candidate list, built in the
// scratch on request (*uniq points into it until the next call uses it).
int build_candidates(dn_volume *v, uint64_t **uniq, int64_t *n_uniq)
{
    *uniq = nullptr;
    *n_uniq = 0;
    const int64_t n = v->cand_n;
    if (n == 0) return DN_OK;
    hipStream_t st = v->stream;
    Bump bump(v->scratch, v->scratch_bytes);
    CandScratch x = carve_cand(bump, n);
    if (!bump.fits()) { set_error("scratch too small for the candidate list"); return DN_E_CAPACITY; }
    int64_t *d_n = v->misc + 3;
    size_t tbytes = x.tmp_bytes;
    DN_HIP(rocprim::radix_sort_keys(x.tmp, tbytes, v->cand, x.sorted, size_t(n), 0, 63, st));
    tbytes = x.tmp_bytes;
    DN_HIP(rocprim::unique(x.tmp, tbytes, x.sorted, x.uniq, d_n, size_t(n), rocprim::equal_to<uint64_t>(), st));
    int rc = read_back(v, d_n, sizeof(int64_t));
    if (rc) return rc;
    *uniq = x.uniq;
    *n_uniq = v->host_stage[0];
    return DN_OK;
}

// Placement of everything a volume keeps in its arena (base == nullptr:
// measure only).  Returns the arena size; with v != nullptr the volume's
// pointers are set.
static size_t volume_layout(const dn_volume_params &p, void *base, dn_volume *v)
{
    const size_t mb = size_t(p.max_blocks), vox = mb * kBlockVox;
    const size_t slots = (size_t(1) << p.hash_cap_log2) + size_t(p.hash_tail);
    Bump b(base, ~size_t(0));
    int32_t *coords = b.take<int32_t>(mb * 4);
    uint64_t *keys = b.take<uint64_t>(mb);
    int32_t *h0 = b.take<int32_t>(slots * 4);
    int32_t *h1 = b.take<int32_t>(slots * 4);
    int32_t *nbr = b.take<int32_t>(mb * kNbr);
    float *f = b.take<float>(vox);
    float *w = b.take<float>(vox);
    float *u = b.take<float>(vox);
    float *ub0 = b.take<float>(vox);
    float *ub1 = b.take<float>(vox);
    float *p0 = b.take<float>(vox * 3);
    float *p1 = b.take<float>(vox * 3);
    uint8_t *emask = b.take<uint8_t>(vox);
    int32_t *order = b.take<int32_t>(mb);
    double *partials = b.take<double>(mb * 2 + 2 * ((mb + 1023) / 1024 + 1) * 2 + 8);
    double *energy2 = b.take<double>(8);
    int64_t *misc = b.take<int64_t>(32);
    uint64_t *cand = b.take<uint64_t>(size_t(p.max_candidates));
    void *u16 = nullptr, *ub16a = nullptr, *ub16b = nullptr, *p16a = nullptr, *p16b = nullptr;
    if (p.state16) {
        u16 = b.take<uint16_t>(vox);
        ub16a = b.take<uint16_t>(vox);
        ub16b = b.take<uint16_t>(vox);
        p16a = b.take<uint16_t>(vox * 3);
        p16b = b.take<uint16_t>(vox * 3);
    }
    // scratch: the largest of the per-call needs
    size_t need = 0;
    auto upd = [&](size_t n) { need = std::max(need, n); };
    {
        Bump m(nullptr, 0);
        carve_frame(m, p.max_points);
        upd(m.off);
    }
    {
        Bump m(nullptr, 0);
        carve_insert(m, std::max<int64_t>(p.max_candidates, 1), p.max_blocks);
        upd(m.off);
    }
    upd(candidates_scratch(std::max<int64_t>(p.max_candidates, 1)));
    upd(masks_scratch(p.max_blocks));
    upd(extract_scratch(p.max_blocks));
    if (p.max_observations > 0) {
        Bump m(nullptr, 0);
        carve_laser(m, p.max_points, p.max_observations);
        upd(m.off);
    }
    upd(size_t(p.max_blocks) * sizeof(int32_t));   // the blocks in view of a fused frame
    char *scratch = b.take<char>(need);
    if (v) {
        v->coords = coords; v->keys = keys; v->hash[0] = h0; v->hash[1] = h1; v->nbr = nbr;
        v->f = f; v->w = w; v->u = u; v->ubar[0] = ub0; v->ubar[1] = ub1; v->p[0] = p0; v->p[1] = p1;
        v->emask = emask; v->order = order; v->partials = partials; v->energy2 = energy2; v->misc = misc;
        v->cand = cand;
        v->u16 = u16; v->ubar16[0] = ub16a; v->ubar16[1] = ub16b; v->p16[0] = p16a; v->p16[1] = p16b;
        v->scratch = scratch;
        v->scratch_bytes = need;
    }
    return (b.off + 255) & ~size_t(255);
}

static bool params_ok(const dn_volume_params *p)
{
    return p && p->voxel_size > 0 && p->mu > 0 && p->max_depth > 0 && p->max_blocks >= 1 &&
           p->hash_cap_log2 >= 4 && p->hash_cap_log2 <= 30 && p->hash_tail >= 0 &&
           (p->state16 == 0 || p->state16 == 1) && p->max_points >= 0 && p->max_candidates >= 0 &&
           p->max_observations >= 0 && p->max_points < (int64_t(1) << 31) &&
           p->max_candidates < (int64_t(1) << 40) && p->max_observations < (int64_t(1) << 32) &&
           std::isfinite(p->voxel_size) && std::isfinite(p->mu) && std::isfinite(p->max_depth);
}

// The rocprim calls' own storage figures at the largest sizes this volume
// can ask for, against the bounds its scratch was sized with.
static int verify_tmp_bounds(dn_volume *v)
{
    const dn_volume_params &p = v->prm;
    hipStream_t st = v->stream;
    const size_t nc = size_t(std::max<int64_t>(p.max_candidates, 1)), mb = size_t(p.max_blocks);
    const size_t np = size_t(std::max<int64_t>(p.max_points, 1)), no = size_t(std::max<int64_t>(p.max_observations, 1));
    struct Q { const char *what; size_t need, have; };
    std::vector<Q> q;
    size_t t = 0;
    int32_t *i32 = nullptr; int64_t *i64 = nullptr; uint64_t *u64 = nullptr; uint32_t *u32 = nullptr;
    uint8_t *u8 = nullptr; double *f64 = nullptr;
    DN_HIP(rocprim::exclusive_scan(nullptr, t, i32, i32, 0, np, rocprim::plus<int32_t>(), st));
    q.push_back({"point scan", t, tmp_light(np)});
    t = 0;
    DN_HIP(rocprim::select(nullptr, t, u64, u8, u64, i64, nc, st));
    q.push_back({"candidate selection", t, tmp_light(nc)});
    t = 0;
    DN_HIP(rocprim::radix_sort_keys(nullptr, t, u64, u64, nc, 0, 63, st));
    q.push_back({"candidate sort", t, tmp_sort(nc, 8)});
    t = 0;
    DN_HIP(rocprim::unique(nullptr, t, u64, u64, i64, nc, rocprim::equal_to<uint64_t>(), st));
    q.push_back({"candidate unique", t, tmp_light(nc)});
    t = 0;
    DN_HIP(rocprim::radix_sort_pairs(nullptr, t, u64, u64, i32, i32, nc, 0, 63, st));
    q.push_back({"candidate sort with positions", t, tmp_sort(nc, 12)});
    t = 0;
    DN_HIP(rocprim::select(nullptr, t, i32, u8, i32, i64, nc, st));
    q.push_back({"first-occurrence selection", t, tmp_light(nc)});
    t = 0;
    DN_HIP(rocprim::radix_sort_keys(nullptr, t, i32, i32, nc, 0, 31, st));
    q.push_back({"position sort", t, tmp_sort(nc, 12)});
    t = 0;
    DN_HIP(rocprim::radix_sort_pairs(nullptr, t, u64, u64, i32, i32, mb, 0, 63, st));
    q.push_back({"key sort", t, tmp_sort(mb, 12)});
    t = 0;
    DN_HIP(rocprim::radix_sort_pairs(nullptr, t, u32, u32, i32, i32, mb, 0, 31, st));
    q.push_back({"bucket sort", t, tmp_sort(mb, 8)});
    t = 0;
    DN_HIP(rocprim::inclusive_scan(nullptr, t, i64, i64, mb, rocprim::maximum<int64_t>(), st));
    q.push_back({"slot scan", t, tmp_light(mb)});
    t = 0;
    DN_HIP(rocprim::exclusive_scan(nullptr, t, i64, i64, int64_t(0), mb + 1, rocprim::plus<int64_t>(), st));
    q.push_back({"extraction scan", t, tmp_light(mb + 1)});
    if (p.max_observations > 0) {
        t = 0;
        DN_HIP(rocprim::exclusive_scan(nullptr, t, i64, i64, int64_t(0), np, rocprim::plus<int64_t>(), st));
        q.push_back({"return scan", t, tmp_light(np)});
        t = 0;
        DN_HIP(rocprim::radix_sort_pairs(nullptr, t, u32, u32, f64, f64, no, 0, 32, st));
        q.push_back({"observation sort", t, tmp_sort(no, 12)});
        t = 0;
        DN_HIP(rocprim::reduce_by_key(nullptr, t, u32, f64, no, u32, f64, u32, rocprim::plus<double>(),
                                      rocprim::equal_to<uint32_t>(), st));
        q.push_back({"observation sums", t, tmp_light(no)});
        t = 0;
        DN_HIP(rocprim::run_length_encode(nullptr, t, u32, no, u32, u32, u32, st));
        q.push_back({"observation counts", t, tmp_light(no)});
    }
    for (const Q &e : q)
        if (e.need > e.have) {
            set_error("rocprim %s needs %zu bytes of storage, the scratch bound is %zu", e.what, e.need, e.have);
            return DN_E_CAPACITY;
        }
    return DN_OK;
}

// Band cells of n points (depth pixels or laser returns): count, scan, check
// the limit, emit into v->cand; then the shared insertion.
template <class Count, class Emit>
static int alloc_points(dn_volume *v, int64_t n, Count count, Emit emit, int32_t *n_new_out)
{
    if (n_new_out) *n_new_out = 0;
    v->cand_n = 0;
    if (n == 0) return DN_OK;
    if (n > v->prm.max_points) {
        set_error("%lld points exceed the volume's max_points %lld", (long long)n, (long long)v->prm.max_points);
        return DN_E_CAPACITY;
    }
    hipStream_t st = v->stream;
    Bump bump(v->scratch, v->scratch_bytes);
    FrameScratch x = carve_frame(bump, n);
    if (!bump.fits()) { set_error("scratch too small for %lld points", (long long)n); return DN_E_CAPACITY; }
    count(x.counts);
    DN_HIP(hipGetLastError());
    size_t tbytes = x.tmp_bytes;
    DN_HIP(rocprim::exclusive_scan(x.tmp, tbytes, x.counts, x.offs, 0, size_t(n), rocprim::plus<int32_t>(), st));
    int32_t pair[2];
    DN_HIP(hipMemcpyAsync(reinterpret_cast<char *>(v->host_stage), x.offs + n - 1, 4, hipMemcpyDeviceToHost, st));
    DN_HIP(hipMemcpyAsync(reinterpret_cast<char *>(v->host_stage) + 4, x.counts + n - 1, 4, hipMemcpyDeviceToHost, st));
    DN_HIP(hipStreamSynchronize(st));
    memcpy(pair, v->host_stage, 8);
    const int64_t total = int64_t(pair[0]) + pair[1];
    if (total == 0) return DN_OK;
    if (total > v->prm.max_candidates) {
        set_error("%lld band cells exceed the volume's max_candidates %lld", (long long)total,
                  (long long)v->prm.max_candidates);
        return DN_E_CAPACITY;
    }
    emit(x.offs, total);
    DN_HIP(hipGetLastError());
    return insert_packed(v, v->cand, total, n_new_out);
}

}  // namespace dn

using namespace dn;

// ================================================================== C ABI
extern "C" {

const char *dn_last_error(void) { return g_err; }

size_t dn_volume_bytes(const dn_volume_params *p)
{
    if (!params_ok(p)) return 0;
    return volume_layout(*p, nullptr, nullptr);
}

int dn_volume_create(const dn_volume_params *p, void *arena, size_t arena_bytes, void *hip_stream, dn_volume **out)
{
    DN_REQUIRE(p && out, "null argument");
    *out = nullptr;
    DN_REQUIRE(p->voxel_size > 0 && p->mu > 0 && p->max_depth > 0, "voxel_size, mu, max_depth must be > 0");
    DN_REQUIRE(p->max_blocks >= 1, "max_blocks must be >= 1");
    DN_REQUIRE(p->hash_cap_log2 >= 4 && p->hash_cap_log2 <= 30, "hash_cap_log2 must be in [4, 30]");
    DN_REQUIRE(p->hash_tail >= 0, "hash_tail must be >= 0");
    DN_REQUIRE(params_ok(p), "bad limits (state16 0/1; max_points, max_candidates, max_observations >= 0 and in range)");
    DN_REQUIRE(arena, "null arena");
    DN_REQUIRE((reinterpret_cast<uintptr_t>(arena) & 255) == 0, "the arena must be 256-byte aligned");
    const size_t need = volume_layout(*p, nullptr, nullptr);
    if (arena_bytes < need) {
        set_error("arena of %zu bytes is short: the volume needs %zu (dn_volume_bytes)", arena_bytes, need);
        return DN_E_CAPACITY;
    }
    dn_volume *v = new dn_volume();
    v->prm = *p;
    v->stream = static_cast<hipStream_t>(hip_stream);
    v->cap_blocks = p->max_blocks;
    v->hash_cap = 1u << p->hash_cap_log2;
    v->hash_slots = int64_t(v->hash_cap) + p->hash_tail;
    v->arena = arena;
    v->arena_bytes = arena_bytes;
    volume_layout(*p, arena, v);
    auto fail = [&](int rc) { delete v; return rc; };
    if (hipGetDevice(&v->device) != hipSuccess) { set_error("hipGetDevice failed"); return fail(DN_E_DEVICE); }
    int rc = verify_tmp_bounds(v);
    if (rc) return fail(rc);
    hipStream_t st = v->stream;
    const int64_t vox = int64_t(v->cap_blocks) * kBlockVox;
    hipLaunchKernelGGL(k_zero_blocks, dim3(grid1(vox)), dim3(256), 0, st, v->f, int64_t(0), v->cap_blocks);
    hipLaunchKernelGGL(k_zero_blocks, dim3(grid1(vox)), dim3(256), 0, st, v->w, int64_t(0), v->cap_blocks);
    hipLaunchKernelGGL(k_fill_empty, dim3(grid1(v->hash_slots)), dim3(256), 0, st,
                       reinterpret_cast<int4 *>(v->hash[0]), v->hash_slots);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        set_error("initialisation failed");
        return fail(DN_E_DEVICE);
    }
    *out = v;
    return DN_OK;
}

void dn_volume_destroy(dn_volume *v)
{
    if (!v) return;
    (void)hipStreamSynchronize(v->stream);
    delete v;
}

int dn_volume_clear(dn_volume *v)
{
    DN_REQUIRE(v, "null volume");
    hipStream_t st = v->stream;
    hipLaunchKernelGGL(k_fill_empty, dim3(grid1(v->hash_slots)), dim3(256), 0, st,
                       reinterpret_cast<int4 *>(v->hash[v->cur_hash]), v->hash_slots);
    DN_HIP(hipGetLastError());
    if (v->nb > 0) {
        hipLaunchKernelGGL(k_zero_blocks, dim3(grid1(v->nb * kBlockVox)), dim3(256), 0, st, v->f, int64_t(0), v->nb);
        hipLaunchKernelGGL(k_zero_blocks, dim3(grid1(v->nb * kBlockVox)), dim3(256), 0, st, v->w, int64_t(0), v->nb);
        DN_HIP(hipGetLastError());
    }
    v->nb = 0;
    v->nb_state = 0;
    v->emask_nb = -1;
    v->cand_n = 0;
    v->state_storage = DN_F32;
    return DN_OK;
}

int dn_set_stream(dn_volume *v, void *hip_stream)
{
    DN_REQUIRE(v, "null volume");
    v->stream = static_cast<hipStream_t>(hip_stream);
    return DN_OK;
}

int64_t dn_num_blocks(const dn_volume *v) { return v ? v->nb : -1; }

int dn_sync(dn_volume *v)
{
    DN_REQUIRE(v, "null volume");
    return volume_sync(v);
}

int dn_alloc_blocks(dn_volume *v, const float *depth, const dn_intrinsics *K, const double T[16],
                    int32_t *n_new_out)
{
    DN_REQUIRE(v && depth, "null argument");
    Geo g;
    int rc = make_geo(v, K, T, g);
    if (rc) return rc;
    hipStream_t st = v->stream;
    const int64_t npx = int64_t(g.W) * g.H;
    return alloc_points(
        v, npx,
        [&](int32_t *counts) {
            hipLaunchKernelGGL(k_dda_count, dim3(grid1(npx)), dim3(256), 0, st, g, depth, counts);
        },
        [&](const int32_t *offs, int64_t total) {
            hipLaunchKernelGGL(k_dda_emit, dim3(grid1(npx)), dim3(256), 0, st, g, depth, offs, v->cand, total);
        },
        n_new_out);
}

static int insert_keys(dn_volume *v, const int32_t *coords, int64_t n, int32_t *n_new_out, bool keep_order)
{
    DN_REQUIRE(v && (coords || n == 0) && n >= 0, "bad argument");
    if (n_new_out) *n_new_out = 0;
    v->cand_n = 0;
    if (n == 0) return DN_OK;
    if (n > v->prm.max_candidates) {
        set_error("%lld keys exceed the volume's max_candidates %lld", (long long)n, (long long)v->prm.max_candidates);
        return DN_E_CAPACITY;
    }
    hipLaunchKernelGGL(k_pack_coords, dim3(grid1(n)), dim3(256), 0, v->stream, coords, n, v->cand);
    DN_HIP(hipGetLastError());
    return insert_packed(v, v->cand, n, n_new_out, keep_order);
}

int dn_insert_blocks(dn_volume *v, const int32_t *coords, int64_t n, int32_t *n_new_out)
{
    return insert_keys(v, coords, n, n_new_out, false);
}

int dn_insert_blocks_ordered(dn_volume *v, const int32_t *coords, int64_t n, int32_t *n_new_out)
{
    DN_REQUIRE(n < (int64_t(1) << 31), "at most 2^31 - 1 keys per call");
    return insert_keys(v, coords, n, n_new_out, true);
}

int dn_fuse_depth(dn_volume *v, const float *depth, const dn_intrinsics *K, const double T[16])
{
    DN_REQUIRE(v && depth, "null argument");
    Geo g;
    int rc = make_geo(v, K, T, g);
    if (rc) return rc;
    if (v->nb == 0) return DN_OK;
    int32_t *list = reinterpret_cast<int32_t *>(v->scratch);
    int32_t *count = reinterpret_cast<int32_t *>(v->misc + kMiscFuseCount);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, v->stream, count);
    hipLaunchKernelGGL(k_cull, dim3(grid1(v->nb)), dim3(256), 0, v->stream, g, v->coords, v->nb, list, count);
    DN_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_fuse_list, dim3(unsigned(std::min<int64_t>(v->nb, kFuseGrid))), dim3(256), 0, v->stream,
                       g, depth, v->coords, list, count, v->f, v->w);
    DN_HIP(hipGetLastError());
    v->emask_nb = -1;
    return DN_OK;
}

int dn_load_fused(dn_volume *v, const float *f, const float *w)
{
    DN_REQUIRE(v && f && w, "null argument");
    if (v->nb == 0) return DN_OK;
    size_t bytes = size_t(v->nb) * kBlockVox * 4;
    DN_HIP(hipMemcpyAsync(v->f, f, bytes, hipMemcpyDeviceToDevice, v->stream));
    DN_HIP(hipMemcpyAsync(v->w, w, bytes, hipMemcpyDeviceToDevice, v->stream));
    v->emask_nb = -1;
    return DN_OK;
}

int dn_alloc_laser(dn_volume *v, const float *pts, int64_t n, const double T[16], int32_t *n_new_out)
{
    DN_REQUIRE(v && (pts || n == 0) && n >= 0, "bad argument");
    LGeo g;
    int rc = make_lgeo(v, T, g);
    if (rc) return rc;
    hipStream_t st = v->stream;
    return alloc_points(
        v, n,
        [&](int32_t *counts) {
            hipLaunchKernelGGL(k_laser_cand_count, dim3(grid1(n)), dim3(256), 0, st, g, pts, n, counts);
        },
        [&](const int32_t *offs, int64_t total) {
            hipLaunchKernelGGL(k_laser_cand_emit, dim3(grid1(n)), dim3(256), 0, st, g, pts, n, offs, v->cand, total);
        },
        n_new_out);
}

int dn_fuse_laser(dn_volume *v, const float *pts, int64_t n, const double T[16])
{
    DN_REQUIRE(v && (pts || n == 0) && n >= 0, "bad argument");
    LGeo g;
    int rc = make_lgeo(v, T, g);
    if (rc) return rc;
    if (n == 0 || v->nb == 0) return DN_OK;
    if (n > v->prm.max_points) {
        set_error("%lld returns exceed the volume's max_points %lld", (long long)n, (long long)v->prm.max_points);
        return DN_E_CAPACITY;
    }
    if (v->prm.max_observations <= 0) { set_error("the volume was created without laser observations"); return DN_E_CAPACITY; }
    DN_REQUIRE(v->nb * int64_t(kBlockVox) < (int64_t(1) << 32), "volume too large for 32-bit voxel keys");
    hipStream_t st = v->stream;
    const int4 *slots = reinterpret_cast<const int4 *>(v->hash[v->cur_hash]);
    Bump bump(v->scratch, v->scratch_bytes);
    LaserScratch x = carve_laser(bump, n, v->prm.max_observations);
    if (!bump.fits()) { set_error("scratch too small for the laser observations"); return DN_E_CAPACITY; }
    hipLaunchKernelGGL(k_laser_obs_count, dim3(grid1(n)), dim3(256), 0, st, g, pts, n, slots, v->hash_slots,
                       v->hash_cap, x.counts);
    DN_HIP(hipGetLastError());
    size_t tbytes = x.tmp_bytes;
    DN_HIP(rocprim::exclusive_scan(x.tmp, tbytes, x.counts, x.offs, int64_t(0), size_t(n),
                                   rocprim::plus<int64_t>(), st));
    DN_HIP(hipMemcpyAsync(v->host_stage, x.offs + n - 1, 8, hipMemcpyDeviceToHost, st));
    DN_HIP(hipMemcpyAsync(v->host_stage + 1, x.counts + n - 1, 8, hipMemcpyDeviceToHost, st));
    DN_HIP(hipStreamSynchronize(st));
    const int64_t m = v->host_stage[0] + v->host_stage[1];
    if (m == 0) return DN_OK;
    if (m > v->prm.max_observations) {
        set_error("%lld laser observations exceed the volume's max_observations %lld", (long long)m,
                  (long long)v->prm.max_observations);
        return DN_E_CAPACITY;
    }
    hipLaunchKernelGGL(k_laser_obs_emit, dim3(grid1(n)), dim3(256), 0, st, g, pts, n, slots, v->hash_slots,
                       v->hash_cap, x.offs, x.k_in, x.v_in, m);
    DN_HIP(hipGetLastError());
    int bits = 1;
    while ((int64_t(1) << bits) < v->nb * int64_t(kBlockVox)) ++bits;
    // sort by voxel, then the sum and the count of each voxel's observations
    // (distinct voxels into k_in / v_in, counts into counts32)
    tbytes = x.tmp_bytes;
    DN_HIP(rocprim::radix_sort_pairs(x.tmp, tbytes, x.k_in, x.k_out, x.v_in, x.v_out, size_t(m), 0, bits, st));
    tbytes = x.tmp_bytes;
    DN_HIP(rocprim::reduce_by_key(x.tmp, tbytes, x.k_out, x.v_out, size_t(m), x.k_in, x.v_in, x.nruns,
                                  rocprim::plus<double>(), rocprim::equal_to<uint32_t>(), st));
    tbytes = x.tmp_bytes;
    DN_HIP(rocprim::run_length_encode(x.tmp, tbytes, x.k_out, size_t(m), x.k_in, x.counts32, x.nruns, st));
    hipLaunchKernelGGL(k_laser_apply, dim3(grid1(m)), dim3(256), 0, st, x.k_in, x.v_in, x.counts32, x.nruns, m,
                       v->f, v->w);
    DN_HIP(hipGetLastError());
    v->emask_nb = -1;
    return DN_OK;
}

}  // extern "C"
