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

int Buf::ensure(size_t need)
{
    if (need <= bytes) return DN_OK;
    if (ptr) { (void)hipFree(ptr); ptr = nullptr; bytes = 0; }
    size_t nb = need + need / 4 + 256;
    DN_HIP(hipMalloc(&ptr, nb));
    bytes = nb;
    return DN_OK;
}

void Buf::release()
{
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

int HostBuf::ensure(size_t need)
{
    if (need <= bytes) return DN_OK;
    if (ptr) { (void)hipHostFree(ptr); ptr = nullptr; bytes = 0; }
    DN_HIP(hipHostMalloc(&ptr, need < 4096 ? 4096 : need, hipHostMallocDefault));
    bytes = need < 4096 ? 4096 : need;
    return DN_OK;
}

void HostBuf::release()
{
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
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

// Grid traversal of one pixel's band over the block grid.  Emits the
// visited block keys through `emit` and returns how many were visited.
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
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (!(fabs(a[i]) < 1e6 && fabs(b[i]) < 1e6)) return 0;
    int64_t k[3], left[3];
    int step[3];
    double tmax[3], tdel[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        k[i] = int64_t(floor(a[i]));
        int64_t e = int64_t(floor(b[i]));
        double dir = b[i] - a[i];
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
    int n = 0;
    for (;;) {
        emit(n, int32_t(k[0]), int32_t(k[1]), int32_t(k[2]));
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

// Insert a packed candidate list (device, n_cand entries, repeats allowed).
// Appends the keys not yet present in ascending order, rebuilds hash +
// neighbours.  The raw list is first filtered against the table, so only
// candidates of new blocks are sorted (after the first frames of a sequence
// almost every candidate is a block that exists); the ascending list of all
// distinct candidates is built from the same raw list only when it is
// extracted (ensure_candidates).
static int insert_packed(dn_volume *v, uint64_t *cand, int64_t n_cand, int32_t *n_new_out)
{
    hipStream_t st = v->stream;
    if (n_new_out) *n_new_out = 0;
    v->last_nuniq = 0;
    v->cand_src = cand;
    v->cand_n = n_cand;
    v->cand_pending = n_cand > 0;
    if (n_cand == 0) return DN_OK;
    int rc;
    // 1) the candidates of blocks not in the table (repeats kept)
    if ((rc = v->s_flags.ensure(n_cand))) return rc;
    if ((rc = v->s_new.ensure(n_cand * sizeof(uint64_t)))) return rc;
    if ((rc = v->s_misc.ensure(64))) return rc;
    int64_t *d_nraw = v->s_misc.as<int64_t>();
    int64_t *d_nnew = d_nraw + 1;
    const int4 *slots = reinterpret_cast<const int4 *>(v->hash[v->cur_hash]);
    hipLaunchKernelGGL(k_flag_unknown, dim3(grid1(n_cand)), dim3(256), 0, st, cand, n_cand, slots,
                       v->hash_slots, v->hash_cap, v->s_flags.as<uint8_t>());
    DN_HIP(hipGetLastError());
    size_t tb = 0;
    DN_HIP(rocprim::select(nullptr, tb, cand, v->s_flags.as<uint8_t>(), v->s_new.as<uint64_t>(), d_nraw,
                           size_t(n_cand), st));
    if ((rc = v->s_tmp.ensure(tb))) return rc;
    size_t tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::select(v->s_tmp.ptr, tbytes, cand, v->s_flags.as<uint8_t>(), v->s_new.as<uint64_t>(),
                           d_nraw, size_t(n_cand), st));
    if ((rc = v->host.ensure(64))) return rc;
    DN_HIP(hipMemcpyAsync(v->host.ptr, d_nraw, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DN_HIP(hipStreamSynchronize(st));
    const int64_t n_raw = v->host.as<int64_t>()[0];
    if (n_raw == 0) return DN_OK;
    // 2) the distinct new keys, ascending
    if ((rc = v->s_sorted.ensure(n_raw * sizeof(uint64_t)))) return rc;
    if ((rc = v->s_newk.ensure(n_raw * sizeof(uint64_t)))) return rc;
    uint64_t *sorted = v->s_sorted.as<uint64_t>();
    uint64_t *newk = v->s_newk.as<uint64_t>();
    size_t t2 = 0;
    tb = 0;
    DN_HIP(rocprim::radix_sort_keys(nullptr, tb, v->s_new.as<uint64_t>(), sorted, size_t(n_raw), 0, 63, st));
    DN_HIP(rocprim::unique(nullptr, t2, sorted, newk, d_nnew, size_t(n_raw), rocprim::equal_to<uint64_t>(), st));
    if ((rc = v->s_tmp.ensure(tb > t2 ? tb : t2))) return rc;
    tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::radix_sort_keys(v->s_tmp.ptr, tbytes, v->s_new.as<uint64_t>(), sorted, size_t(n_raw), 0, 63,
                                    st));
    tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::unique(v->s_tmp.ptr, tbytes, sorted, newk, d_nnew, size_t(n_raw), rocprim::equal_to<uint64_t>(),
                           st));
    DN_HIP(hipMemcpyAsync(v->host.ptr, d_nnew, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DN_HIP(hipStreamSynchronize(st));
    const int64_t n_new = v->host.as<int64_t>()[0];
    if (v->nb + n_new > v->cap_blocks) {
        set_error("block pool full: %lld + %lld new blocks > max_blocks %lld", (long long)v->nb,
                  (long long)n_new, (long long)v->cap_blocks);
        return DN_E_CAPACITY;
    }
    // 3) tentatively append (beyond nb; not committed until the hash fits)
    const int64_t nb_old = v->nb, nb_new = v->nb + n_new;
    hipLaunchKernelGGL(k_append, dim3(grid1(n_new)), dim3(256), 0, st, newk, n_new, nb_old, v->coords, v->keys);
    DN_HIP(hipGetLastError());
    // 4) canonical table: sort (key -> id), then stable sort by bucket
    if ((rc = v->s_vals.ensure(nb_new * sizeof(int32_t)))) return rc;
    if ((rc = v->s_vals2.ensure(nb_new * sizeof(int32_t)))) return rc;
    if ((rc = v->s_home.ensure(nb_new * sizeof(uint32_t)))) return rc;
    if ((rc = v->s_home2.ensure(nb_new * sizeof(uint32_t)))) return rc;
    if ((rc = v->s_pos.ensure(nb_new * sizeof(int64_t) * 2))) return rc;
    if ((rc = v->s_cand2.ensure(nb_new * sizeof(uint64_t)))) return rc;
    int32_t *ids0 = v->s_vals.as<int32_t>();
    int32_t *ids1 = v->s_vals2.as<int32_t>();
    uint64_t *ksorted = v->s_cand2.as<uint64_t>();
    uint32_t *home = v->s_home.as<uint32_t>();
    uint32_t *home2 = v->s_home2.as<uint32_t>();
    int64_t *dm = v->s_pos.as<int64_t>();
    int64_t *runmax = dm + nb_new;
    hipLaunchKernelGGL(k_iota, dim3(grid1(nb_new)), dim3(256), 0, st, ids0, nb_new);
    DN_HIP(hipGetLastError());
    tb = 0;
    DN_HIP(rocprim::radix_sort_pairs(nullptr, tb, v->keys, ksorted, ids0, ids1, size_t(nb_new), 0, 63, st));
    const int hbits = bits_for(v->hash_cap - 1);
    t2 = 0;
    DN_HIP(rocprim::radix_sort_pairs(nullptr, t2, home, home2, ids1, ids0, size_t(nb_new), 0, hbits, st));
    tb = tb > t2 ? tb : t2;
    t2 = 0;
    DN_HIP(rocprim::inclusive_scan(nullptr, t2, dm, runmax, size_t(nb_new), rocprim::maximum<int64_t>(), st));
    tb = tb > t2 ? tb : t2;
    if ((rc = v->s_tmp.ensure(tb))) return rc;
    tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::radix_sort_pairs(v->s_tmp.ptr, tbytes, v->keys, ksorted, ids0, ids1, size_t(nb_new), 0, 63, st));
    hipLaunchKernelGGL(k_bucket_of_keys, dim3(grid1(nb_new)), dim3(256), 0, st, ksorted, nb_new, v->hash_cap, home);
    DN_HIP(hipGetLastError());
    tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::radix_sort_pairs(v->s_tmp.ptr, tbytes, home, home2, ids1, ids0, size_t(nb_new), 0, hbits, st));
    hipLaunchKernelGGL(k_home_minus_rank, dim3(grid1(nb_new)), dim3(256), 0, st, home2, nb_new, dm);
    DN_HIP(hipGetLastError());
    tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::inclusive_scan(v->s_tmp.ptr, tbytes, dm, runmax, size_t(nb_new), rocprim::maximum<int64_t>(), st));
    int other = 1 - v->cur_hash;
    int4 *dst = reinterpret_cast<int4 *>(v->hash[other]);
    int32_t *d_ovf = reinterpret_cast<int32_t *>(d_nraw + 2);
    DN_HIP(hipMemsetAsync(d_ovf, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_fill_empty, dim3(grid1(v->hash_slots)), dim3(256), 0, st, dst, v->hash_slots);
    DN_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scatter_slots, dim3(grid1(nb_new)), dim3(256), 0, st, runmax, ids0, v->coords, nb_new,
                       v->hash_slots, dst, d_ovf);
    DN_HIP(hipGetLastError());
    DN_HIP(hipMemcpyAsync(v->host.ptr, d_ovf, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    DN_HIP(hipStreamSynchronize(st));
    if (*v->host.as<int32_t>() != 0) {
        set_error("hash table full: %lld keys do not fit 2^%d buckets + %d tail slots", (long long)nb_new,
                  v->prm.hash_cap_log2, v->prm.hash_tail);
        return DN_E_CAPACITY;
    }
    // 5) commit: new table, zeroed fields of the new blocks, neighbours
    v->cur_hash = other;
    float *fields[] = {v->f, v->w, v->u, v->ubar[0], v->ubar[1]};
    for (float *a : fields) {
        hipLaunchKernelGGL(k_zero_blocks, dim3(grid1(n_new * kBlockVox)), dim3(256), 0, st, a, nb_old, n_new);
        DN_HIP(hipGetLastError());
    }
    for (int pp = 0; pp < 2; ++pp)
        for (int a = 0; a < 3; ++a) {
            hipLaunchKernelGGL(k_zero_blocks, dim3(grid1(n_new * kBlockVox)), dim3(256), 0, st,
                               v->p[pp] + size_t(a) * v->cap_blocks * kBlockVox, nb_old, n_new);
            DN_HIP(hipGetLastError());
        }
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
__global__ void k_fuse(Geo g, const float *__restrict__ depth, const int32_t *__restrict__ coords,
                       int64_t nb, float *__restrict__ f, float *__restrict__ w)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nb * kBlockVox) return;
    int64_t b = i >> 9;
    int vx = int(i & 7), vy = int((i >> 3) & 7), vz = int((i >> 6) & 7);
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
    float wo = w[i];
    float wn = wo + 1.0f;
    f[i] = (float(psi) + wo * f[i]) / wn;
    w[i] = wn;
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

// Amanatides-Woo traversal of a -> b on the unit grid (the allocation
// traversal: ties x before y before z, only axes with steps left).
template <class Emit>
__device__ int64_t walk_segment(const double a[3], const double b[3], Emit emit)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (!(fabs(a[i]) < 1e9 && fabs(b[i]) < 1e9)) return 0;
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
    return walk_segment(a, b, emit);
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
    walk_segment(a, b, [&](int64_t, int64_t x, int64_t y, int64_t z) {
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

// The ascending distinct keys of the last candidate list, in s_uniq
// (last_nuniq of them), built on first request.
int ensure_candidates(dn_volume *v)
{
    if (!v->cand_pending) return DN_OK;
    hipStream_t st = v->stream;
    const int64_t n = v->cand_n;
    int rc;
    if ((rc = v->s_sorted.ensure(n * sizeof(uint64_t)))) return rc;
    if ((rc = v->s_uniq.ensure(n * sizeof(uint64_t)))) return rc;
    if ((rc = v->s_misc.ensure(64))) return rc;
    int64_t *d_n = v->s_misc.as<int64_t>() + 3;
    uint64_t *sorted = v->s_sorted.as<uint64_t>();
    size_t tb = 0, t2 = 0;
    DN_HIP(rocprim::radix_sort_keys(nullptr, tb, v->cand_src, sorted, size_t(n), 0, 63, st));
    DN_HIP(rocprim::unique(nullptr, t2, sorted, v->s_uniq.as<uint64_t>(), d_n, size_t(n),
                           rocprim::equal_to<uint64_t>(), st));
    if ((rc = v->s_tmp.ensure(tb > t2 ? tb : t2))) return rc;
    size_t tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::radix_sort_keys(v->s_tmp.ptr, tbytes, v->cand_src, sorted, size_t(n), 0, 63, st));
    tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::unique(v->s_tmp.ptr, tbytes, sorted, v->s_uniq.as<uint64_t>(), d_n, size_t(n),
                           rocprim::equal_to<uint64_t>(), st));
    if ((rc = v->host.ensure(64))) return rc;
    DN_HIP(hipMemcpyAsync(v->host.ptr, d_n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    DN_HIP(hipStreamSynchronize(st));
    v->last_nuniq = v->host.as<int64_t>()[0];
    v->cand_pending = false;
    return DN_OK;
}

}  // namespace dn

using namespace dn;

// ================================================================== C ABI
extern "C" {

const char *dn_last_error(void) { return g_err; }

int dn_volume_create(const dn_volume_params *p, void *hip_stream, dn_volume **out)
{
    DN_REQUIRE(p && out, "null argument");
    *out = nullptr;
    DN_REQUIRE(p->voxel_size > 0 && p->mu > 0 && p->max_depth > 0, "voxel_size, mu, max_depth must be > 0");
    DN_REQUIRE(p->max_blocks >= 1, "max_blocks must be >= 1");
    DN_REQUIRE(p->hash_cap_log2 >= 4 && p->hash_cap_log2 <= 30, "hash_cap_log2 must be in [4, 30]");
    DN_REQUIRE(p->hash_tail >= 0, "hash_tail must be >= 0");
    dn_volume *v = new dn_volume();
    v->prm = *p;
    v->stream = static_cast<hipStream_t>(hip_stream);
    v->cap_blocks = p->max_blocks;
    v->hash_cap = 1u << p->hash_cap_log2;
    v->hash_slots = int64_t(v->hash_cap) + p->hash_tail;
    auto fail = [&](int rc) { dn_volume_destroy(v); return rc; };
    if (hipGetDevice(&v->device) != hipSuccess) { set_error("hipGetDevice failed"); return fail(DN_E_DEVICE); }
    const size_t vox = size_t(v->cap_blocks) * kBlockVox;
    struct { void **ptr; size_t bytes; } allocs[] = {
        {(void **)&v->coords, size_t(v->cap_blocks) * 16},
        {(void **)&v->keys, size_t(v->cap_blocks) * 8},
        {(void **)&v->hash[0], size_t(v->hash_slots) * 16},
        {(void **)&v->hash[1], size_t(v->hash_slots) * 16},
        {(void **)&v->nbr, size_t(v->cap_blocks) * kNbr * 4},
        {(void **)&v->f, vox * 4},
        {(void **)&v->w, vox * 4},
        {(void **)&v->u, vox * 4},
        {(void **)&v->ubar[0], vox * 4},
        {(void **)&v->ubar[1], vox * 4},
        {(void **)&v->p[0], vox * 12},
        {(void **)&v->p[1], vox * 12},
        {(void **)&v->emask, vox},
        {(void **)&v->order, size_t(v->cap_blocks) * 4},
        {(void **)&v->partials, size_t(v->cap_blocks) * 16 + 2 * (size_t((v->cap_blocks + 1023) / 1024) + 1) * 16 + 64},
        {(void **)&v->energy2, 64},
    };
    for (auto &a : allocs) {
        if (hipMalloc(a.ptr, a.bytes) != hipSuccess) {
            set_error("hipMalloc of %zu bytes failed", a.bytes);
            return fail(DN_E_DEVICE);
        }
    }
    hipStream_t st = v->stream;
    if (hipMemsetAsync(v->f, 0, vox * 4, st) != hipSuccess || hipMemsetAsync(v->w, 0, vox * 4, st) != hipSuccess) {
        set_error("hipMemsetAsync failed");
        return fail(DN_E_DEVICE);
    }
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
    void *ptrs[] = {v->coords, v->keys, v->hash[0], v->hash[1], v->nbr, v->f, v->w, v->u,
                    v->ubar[0], v->ubar[1], v->p[0], v->p[1], v->emask, v->order, v->partials,
                    v->energy2, v->u16, v->ubar16[0], v->ubar16[1], v->p16[0], v->p16[1]};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    dn::Buf *bufs[] = {&v->s_cand, &v->s_cand2, &v->s_counts, &v->s_offsets, &v->s_tmp, &v->s_uniq,
                       &v->s_flags, &v->s_new, &v->s_sorted, &v->s_vals, &v->s_vals2, &v->s_home,
                       &v->s_home2, &v->s_pos, &v->s_misc, &v->s_laser, &v->s_newk};
    for (auto *b : bufs) b->release();
    v->host.release();
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
    v->last_nuniq = 0;
    v->cand_pending = false;
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
    if (n_new_out) *n_new_out = 0;
    hipStream_t st = v->stream;
    const int64_t npx = int64_t(g.W) * g.H;
    if ((rc = v->s_counts.ensure(npx * 4))) return rc;
    if ((rc = v->s_offsets.ensure(npx * 4 + 8))) return rc;
    int32_t *counts = v->s_counts.as<int32_t>();
    int32_t *offs = v->s_offsets.as<int32_t>();
    hipLaunchKernelGGL(k_dda_count, dim3(grid1(npx)), dim3(256), 0, st, g, depth, counts);
    DN_HIP(hipGetLastError());
    size_t tb = 0;
    DN_HIP(rocprim::exclusive_scan(nullptr, tb, counts, offs, 0, size_t(npx), rocprim::plus<int32_t>(), st));
    if ((rc = v->s_tmp.ensure(tb))) return rc;
    size_t tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::exclusive_scan(v->s_tmp.ptr, tbytes, counts, offs, 0, size_t(npx), rocprim::plus<int32_t>(), st));
    if ((rc = v->host.ensure(64))) return rc;
    DN_HIP(hipMemcpyAsync(v->host.as<int32_t>(), offs + npx - 1, 4, hipMemcpyDeviceToHost, st));
    DN_HIP(hipMemcpyAsync(v->host.as<int32_t>() + 1, counts + npx - 1, 4, hipMemcpyDeviceToHost, st));
    DN_HIP(hipStreamSynchronize(st));
    int64_t total = int64_t(v->host.as<int32_t>()[0]) + v->host.as<int32_t>()[1];
    if (total == 0) { v->last_nuniq = 0; v->cand_pending = false; return DN_OK; }
    v->cand_pending = false;
    v->last_nuniq = 0;
    if ((rc = v->s_cand.ensure(total * 8))) return rc;
    hipLaunchKernelGGL(k_dda_emit, dim3(grid1(npx)), dim3(256), 0, st, g, depth, offs, v->s_cand.as<uint64_t>(), total);
    DN_HIP(hipGetLastError());
    return insert_packed(v, v->s_cand.as<uint64_t>(), total, n_new_out);
}

int dn_insert_blocks(dn_volume *v, const int32_t *coords, int64_t n, int32_t *n_new_out)
{
    DN_REQUIRE(v && (coords || n == 0) && n >= 0, "bad argument");
    if (n_new_out) *n_new_out = 0;
    if (n == 0) return DN_OK;
    int rc;
    v->cand_pending = false;
    v->last_nuniq = 0;
    if ((rc = v->s_cand.ensure(n * 8))) return rc;
    hipLaunchKernelGGL(k_pack_coords, dim3(grid1(n)), dim3(256), 0, v->stream, coords, n, v->s_cand.as<uint64_t>());
    DN_HIP(hipGetLastError());
    return insert_packed(v, v->s_cand.as<uint64_t>(), n, n_new_out);
}

int dn_fuse_depth(dn_volume *v, const float *depth, const dn_intrinsics *K, const double T[16])
{
    DN_REQUIRE(v && depth, "null argument");
    Geo g;
    int rc = make_geo(v, K, T, g);
    if (rc) return rc;
    if (v->nb == 0) return DN_OK;
    hipLaunchKernelGGL(k_fuse, dim3(grid1(v->nb * kBlockVox)), dim3(256), 0, v->stream, g, depth, v->coords,
                       v->nb, v->f, v->w);
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
    if (n_new_out) *n_new_out = 0;
    if (n == 0) { v->last_nuniq = 0; v->cand_pending = false; return DN_OK; }
    DN_REQUIRE(n < (int64_t(1) << 31), "too many returns in one scan");
    hipStream_t st = v->stream;
    if ((rc = v->s_counts.ensure(n * 4))) return rc;
    if ((rc = v->s_offsets.ensure(n * 4 + 8))) return rc;
    int32_t *counts = v->s_counts.as<int32_t>();
    int32_t *offs = v->s_offsets.as<int32_t>();
    hipLaunchKernelGGL(k_laser_cand_count, dim3(grid1(n)), dim3(256), 0, st, g, pts, n, counts);
    DN_HIP(hipGetLastError());
    size_t tb = 0;
    DN_HIP(rocprim::exclusive_scan(nullptr, tb, counts, offs, 0, size_t(n), rocprim::plus<int32_t>(), st));
    if ((rc = v->s_tmp.ensure(tb))) return rc;
    size_t tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::exclusive_scan(v->s_tmp.ptr, tbytes, counts, offs, 0, size_t(n), rocprim::plus<int32_t>(), st));
    if ((rc = v->host.ensure(64))) return rc;
    DN_HIP(hipMemcpyAsync(v->host.as<int32_t>(), offs + n - 1, 4, hipMemcpyDeviceToHost, st));
    DN_HIP(hipMemcpyAsync(v->host.as<int32_t>() + 1, counts + n - 1, 4, hipMemcpyDeviceToHost, st));
    DN_HIP(hipStreamSynchronize(st));
    const int64_t total = int64_t(v->host.as<int32_t>()[0]) + v->host.as<int32_t>()[1];
    if (total == 0) { v->last_nuniq = 0; v->cand_pending = false; return DN_OK; }
    v->cand_pending = false;
    v->last_nuniq = 0;
    if ((rc = v->s_cand.ensure(total * 8))) return rc;
    hipLaunchKernelGGL(k_laser_cand_emit, dim3(grid1(n)), dim3(256), 0, st, g, pts, n, offs,
                       v->s_cand.as<uint64_t>(), total);
    DN_HIP(hipGetLastError());
    return insert_packed(v, v->s_cand.as<uint64_t>(), total, n_new_out);
}

int dn_fuse_laser(dn_volume *v, const float *pts, int64_t n, const double T[16])
{
    DN_REQUIRE(v && (pts || n == 0) && n >= 0, "bad argument");
    LGeo g;
    int rc = make_lgeo(v, T, g);
    if (rc) return rc;
    if (n == 0 || v->nb == 0) return DN_OK;
    DN_REQUIRE(v->nb * int64_t(kBlockVox) < (int64_t(1) << 32), "volume too large for 32-bit voxel keys");
    hipStream_t st = v->stream;
    const int4 *slots = reinterpret_cast<const int4 *>(v->hash[v->cur_hash]);
    if ((rc = v->s_counts.ensure(n * 8))) return rc;
    if ((rc = v->s_offsets.ensure(n * 8 + 8))) return rc;
    int64_t *counts = v->s_counts.as<int64_t>();
    int64_t *offs = v->s_offsets.as<int64_t>();
    hipLaunchKernelGGL(k_laser_obs_count, dim3(grid1(n)), dim3(256), 0, st, g, pts, n, slots, v->hash_slots,
                       v->hash_cap, counts);
    DN_HIP(hipGetLastError());
    size_t tb = 0;
    DN_HIP(rocprim::exclusive_scan(nullptr, tb, counts, offs, int64_t(0), size_t(n), rocprim::plus<int64_t>(), st));
    if ((rc = v->s_tmp.ensure(tb))) return rc;
    size_t tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::exclusive_scan(v->s_tmp.ptr, tbytes, counts, offs, int64_t(0), size_t(n),
                                   rocprim::plus<int64_t>(), st));
    if ((rc = v->host.ensure(64))) return rc;
    DN_HIP(hipMemcpyAsync(v->host.as<int64_t>(), offs + n - 1, 8, hipMemcpyDeviceToHost, st));
    DN_HIP(hipMemcpyAsync(v->host.as<int64_t>() + 1, counts + n - 1, 8, hipMemcpyDeviceToHost, st));
    DN_HIP(hipStreamSynchronize(st));
    const int64_t m = v->host.as<int64_t>()[0] + v->host.as<int64_t>()[1];
    if (m == 0) return DN_OK;
    DN_REQUIRE(m < (int64_t(1) << 32), "too many observations in one scan");
    // keys, values, their sorted copies, the counts and the run count
    if ((rc = v->s_laser.ensure(size_t(m) * 48 + 1024))) return rc;
    uint32_t *k_in = reinterpret_cast<uint32_t *>(v->s_laser.ptr);
    uint32_t *k_out = k_in + m;
    double *v_in = reinterpret_cast<double *>(static_cast<char *>(v->s_laser.ptr) + ((size_t(m) * 8 + 255) / 256) * 256);
    double *v_out = v_in + m;
    hipLaunchKernelGGL(k_laser_obs_emit, dim3(grid1(n)), dim3(256), 0, st, g, pts, n, slots, v->hash_slots,
                       v->hash_cap, offs, k_in, v_in, m);
    DN_HIP(hipGetLastError());
    int bits = 1;
    while ((int64_t(1) << bits) < v->nb * int64_t(kBlockVox)) ++bits;
    // sort by voxel, then the sum and the count of each voxel's observations
    // (distinct voxels into k_in / v_in, counts after the sorted values)
    uint32_t *counts32 = reinterpret_cast<uint32_t *>(v_out + m);
    uint32_t *nruns = counts32 + ((m + 63) / 64) * 64;
    size_t t1 = 0, t2 = 0, t3 = 0;
    DN_HIP(rocprim::radix_sort_pairs(nullptr, t1, k_in, k_out, v_in, v_out, size_t(m), 0, bits, st));
    DN_HIP(rocprim::reduce_by_key(nullptr, t2, k_out, v_out, size_t(m), k_in, v_in, nruns, rocprim::plus<double>(),
                                  rocprim::equal_to<uint32_t>(), st));
    DN_HIP(rocprim::run_length_encode(nullptr, t3, k_out, size_t(m), k_in, counts32, nruns, st));
    if ((rc = v->s_tmp.ensure(std::max(t1, std::max(t2, t3))))) return rc;
    tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::radix_sort_pairs(v->s_tmp.ptr, tbytes, k_in, k_out, v_in, v_out, size_t(m), 0, bits, st));
    tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::reduce_by_key(v->s_tmp.ptr, tbytes, k_out, v_out, size_t(m), k_in, v_in, nruns,
                                  rocprim::plus<double>(), rocprim::equal_to<uint32_t>(), st));
    tbytes = v->s_tmp.bytes;
    DN_HIP(rocprim::run_length_encode(v->s_tmp.ptr, tbytes, k_out, size_t(m), k_in, counts32, nruns, st));
    hipLaunchKernelGGL(k_laser_apply, dim3(grid1(m)), dim3(256), 0, st, k_in, v_in, counts32, nruns, m, v->f, v->w);
    DN_HIP(hipGetLastError());
    v->emask_nb = -1;
    return DN_OK;
}

}  // extern "C"
