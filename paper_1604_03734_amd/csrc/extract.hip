// Extraction of the volume's parts and of the zero-crossing surface of u
// (the model handed to consumers, Section II / Fig. 2 of the paper).
#include <cstring>
#include <rocprim/rocprim.hpp>

#include "dn_internal.h"

namespace dn {

static inline unsigned grid1(int64_t n, int bs = 256) { return unsigned((n + bs - 1) / bs); }

__device__ __forceinline__ int64_t nb_index(const int32_t *nb27, int hx, int hy, int hz)
{
    int dx = hx < 0 ? -1 : (hx > 7 ? 1 : 0);
    int dy = hy < 0 ? -1 : (hy > 7 ? 1 : 0);
    int dz = hz < 0 ? -1 : (hz > 7 ? 1 : 0);
    int32_t id = nb27[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
    if (id < 0) return -1;
    return int64_t(id) * kBlockVox + ((hx - 8 * dx) + 8 * (hy - 8 * dy) + 64 * (hz - 8 * dz));
}

// Number of crossings of voxel g (0..3): axes a with both g and g + e_a
// observed and u(g) < 0 differing from u(g + e_a) < 0.
__device__ __forceinline__ int crossing_bits(const int32_t *nb27, const float *u, const uint8_t *emask,
                                             int64_t gi, int lx, int ly, int lz, float u0[4])
{
    uint8_t m = emask[gi];
    int bits = 0;
    u0[0] = u[gi];
    if (!(m & 1)) return 0;
    const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int a = 0; a < 3; ++a) {
        if (!(m & (2 << a))) continue;
        int64_t j = nb_index(nb27, lx + off[a][0], ly + off[a][1], lz + off[a][2]);
        float u1 = u[j];
        u0[1 + a] = u1;
        if ((u0[0] < 0.0f) != (u1 < 0.0f)) bits |= 1 << a;
    }
    return bits;
}

__global__ __launch_bounds__(512) void k_surface_count(int64_t nb, const int32_t *__restrict__ nbr,
                                                       const uint8_t *__restrict__ emask,
                                                       const float *__restrict__ u, int64_t *__restrict__ counts)
{
    __shared__ int wsum[8];
    const int64_t b = blockIdx.x;
    const int t = threadIdx.x;
    float uu[4];
    int bits = crossing_bits(nbr + b * kNbr, u, emask, b * kBlockVox + t, t & 7, (t >> 3) & 7, t >> 6, uu);
    int c = __popc(bits);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((t & 63) == 0) wsum[t >> 6] = c;
    __syncthreads();
    if (t == 0) {
        int s = 0;
        for (int i = 0; i < 8; ++i) s += wsum[i];
        counts[b] = s;
    }
}

__global__ __launch_bounds__(512) void k_surface_write(int64_t nb, const int32_t *__restrict__ coords,
                                                       const int32_t *__restrict__ nbr,
                                                       const uint8_t *__restrict__ emask,
                                                       const float *__restrict__ u,
                                                       const int64_t *__restrict__ offsets, double s,
                                                       float *__restrict__ out)
{
    __shared__ int scan[512];
    const int64_t b = blockIdx.x;
    const int t = threadIdx.x, lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
    float uu[4];
    int bits = crossing_bits(nbr + b * kNbr, u, emask, b * kBlockVox + t, lx, ly, lz, uu);
    // exclusive scan of the per-voxel counts in voxel order (Hillis-Steele)
    scan[t] = __popc(bits);
    __syncthreads();
    for (int d = 1; d < 512; d <<= 1) {
        int v = t >= d ? scan[t - d] : 0;
        __syncthreads();
        scan[t] += v;
        __syncthreads();
    }
    int64_t pos = offsets[b] + scan[t] - __popc(bits);
    const int l[3] = {lx, ly, lz};
    for (int a = 0; a < 3; ++a) {
        if (!(bits & (1 << a))) continue;
        double u0 = uu[0], u1 = uu[1 + a];
        double tt = u0 / (u0 - u1);
        for (int i = 0; i < 3; ++i) {
            double c = (double(8 * coords[4 * b + i] + l[i]) + 0.5) * s;
            out[3 * pos + i] = float(c + (i == a ? tt * s : 0.0));
        }
        ++pos;
    }
}

// ------------------------------------------------------------------ mesh
// Zero level set of u as triangles (Section II; Tables III and IV report
// the area of this surface).  Cubes are voxel g and g + {0,1}^3 (corner
// k = x + 2y + 4z), meshed only when all eight corners are observed (bit 0
// of the edge mask).  Each cube is cut into six tetrahedra along its main
// diagonal, corners 0, e_a0, e_a0 + e_a1, 7 for the axis orders below, so
// neighbouring cubes cut their shared faces alike.  One vertex alone on
// its side of zero gives the triangle on its three edges (increasing
// tetrahedron order); two and two (negative a < b, positive c < d) give
// (ac, ad, bd) and (ac, bd, bc).  Edge points are taken from the corner
// with the smaller k, so a shared edge is computed identically everywhere;
// a triangle is turned when its normal points against r = n_neg *
// sum(positive offsets) - n_pos * sum(negative offsets).  Double precision
// throughout; the output rounds to float.  Order: pool id, voxel,
// tetrahedron, triangle.
__constant__ int kTetAxes[6][2] = {{0, 1}, {0, 2}, {1, 0}, {1, 2}, {2, 0}, {2, 1}};

struct Cube {
    double u[8];
};

__device__ __forceinline__ bool cube_load(const int32_t *nb27, const float *u, const uint8_t *emask, int lx, int ly,
                                          int lz, Cube &c)
{
    for (int k = 0; k < 8; ++k) {
        const int64_t j = nb_index(nb27, lx + (k & 1), ly + ((k >> 1) & 1), lz + ((k >> 2) & 1));
        if (j < 0 || !(emask[j] & 1)) return false;
        c.u[k] = double(u[j]);
    }
    return true;
}

__device__ __forceinline__ int cube_count(const Cube &c)
{
    int n = 0;
    for (int tt = 0; tt < 6; ++tt) {
        const int a0 = kTetAxes[tt][0], a1 = kTetAxes[tt][1];
        const int kk[4] = {0, 1 << a0, (1 << a0) | (1 << a1), 7};
        int nneg = 0;
        for (int q = 0; q < 4; ++q) nneg += c.u[kk[q]] < 0.0;
        n += (nneg == 1 || nneg == 3) ? 1 : (nneg == 2 ? 2 : 0);
    }
    return n;
}

// Visit the cube's triangles in order: fn(A, B, C) with the oriented
// vertices (world metres).
template <class F>
__device__ __forceinline__ void cube_triangles(const Cube &c, const int32_t *c4, int lx, int ly, int lz, double s,
                                               F fn)
{
    const int l[3] = {lx, ly, lz};
    auto pos = [&](int k, int comp) {
        return (double(8 * c4[comp] + l[comp] + ((k >> comp) & 1)) + 0.5) * s;
    };
    auto edge = [&](int ki, int kj, double out[3]) {
        if (ki > kj) { const int x = ki; ki = kj; kj = x; }
        const double t = c.u[ki] / (c.u[ki] - c.u[kj]);
        for (int comp = 0; comp < 3; ++comp) {
            const double pi = pos(ki, comp), pj = pos(kj, comp);
            out[comp] = pi + t * (pj - pi);
        }
    };
    for (int tt = 0; tt < 6; ++tt) {
        const int a0 = kTetAxes[tt][0], a1 = kTetAxes[tt][1];
        const int kk[4] = {0, 1 << a0, (1 << a0) | (1 << a1), 7};
        int neg[4], nneg = 0;
        for (int q = 0; q < 4; ++q) { neg[q] = c.u[kk[q]] < 0.0; nneg += neg[q]; }
        if (nneg == 0 || nneg == 4) continue;
        double r[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < 4; ++q)
            for (int comp = 0; comp < 3; ++comp) {
                const double oc = double((kk[q] >> comp) & 1);
                r[comp] += neg[q] ? -double(4 - nneg) * oc : double(nneg) * oc;
            }
        auto tri = [&](int e0a, int e0b, int e1a, int e1b, int e2a, int e2b) {
            double A[3], B[3], C[3];
            edge(kk[e0a], kk[e0b], A);
            edge(kk[e1a], kk[e1b], B);
            edge(kk[e2a], kk[e2b], C);
            const double ab[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
            const double ac[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
            const double nx = ab[1] * ac[2] - ab[2] * ac[1];
            const double ny = ab[2] * ac[0] - ab[0] * ac[2];
            const double nz = ab[0] * ac[1] - ab[1] * ac[0];
            const bool flip = (nx * r[0] + ny * r[1]) + nz * r[2] < 0.0;
            const double area = 0.5 * sqrt((nx * nx + ny * ny) + nz * nz);
            if (flip) fn(A, C, B, area);
            else fn(A, B, C, area);
        };
        if (nneg == 1 || nneg == 3) {
            int odd = 0, j[3], m = 0;
            for (int q = 0; q < 4; ++q)
                if (neg[q] == (nneg == 1)) odd = q;
            for (int q = 0; q < 4; ++q)
                if (q != odd) j[m++] = q;
            tri(odd, j[0], odd, j[1], odd, j[2]);
        } else {
            int ng[2], ps[2], mn = 0, mp = 0;
            for (int q = 0; q < 4; ++q) {
                if (neg[q]) ng[mn++] = q;
                else ps[mp++] = q;
            }
            tri(ng[0], ps[0], ng[0], ps[1], ng[1], ps[1]);
            tri(ng[0], ps[0], ng[1], ps[1], ng[1], ps[0]);
        }
    }
}

__global__ __launch_bounds__(512) void k_mesh_count(int64_t nb, const int32_t *__restrict__ nbr,
                                                    const uint8_t *__restrict__ emask, const float *__restrict__ u,
                                                    int64_t *__restrict__ counts)
{
    __shared__ int wsum[8];
    const int64_t b = blockIdx.x;
    const int t = threadIdx.x;
    Cube c;
    int n = cube_load(nbr + b * kNbr, u, emask, t & 7, (t >> 3) & 7, t >> 6, c) ? cube_count(c) : 0;
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    if ((t & 63) == 0) wsum[t >> 6] = n;
    __syncthreads();
    if (t == 0) {
        int sum = 0;
        for (int i = 0; i < 8; ++i) sum += wsum[i];
        counts[b] = sum;
    }
}

__global__ __launch_bounds__(512) void k_mesh_write(int64_t nb, const int32_t *__restrict__ coords,
                                                    const int32_t *__restrict__ nbr,
                                                    const uint8_t *__restrict__ emask, const float *__restrict__ u,
                                                    const int64_t *__restrict__ offsets, double s,
                                                    float *__restrict__ out)
{
    __shared__ int scan[512];
    const int64_t b = blockIdx.x;
    const int t = threadIdx.x, lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
    Cube c;
    const bool ok = cube_load(nbr + b * kNbr, u, emask, lx, ly, lz, c);
    const int n = ok ? cube_count(c) : 0;
    scan[t] = n;
    __syncthreads();
    for (int d = 1; d < 512; d <<= 1) {
        const int v = t >= d ? scan[t - d] : 0;
        __syncthreads();
        scan[t] += v;
        __syncthreads();
    }
    if (!ok || n == 0) return;
    int64_t pos = offsets[b] + scan[t] - n;
    cube_triangles(c, coords + 4 * b, lx, ly, lz, s, [&](const double *A, const double *B, const double *C, double) {
        float *o = out + 9 * pos;
        for (int i = 0; i < 3; ++i) {
            o[i] = float(A[i]);
            o[3 + i] = float(B[i]);
            o[6 + i] = float(C[i]);
        }
        ++pos;
    });
}

// Per-block (area, triangle count) pairs, float64, fixed order: lanes by
// xor butterflies, then the 8 wave sums in wave order.
__global__ __launch_bounds__(512) void k_mesh_area(int64_t nb, const int32_t *__restrict__ coords,
                                                   const int32_t *__restrict__ nbr,
                                                   const uint8_t *__restrict__ emask, const float *__restrict__ u,
                                                   double s, double *__restrict__ partials)
{
    __shared__ double wa[8], wn[8];
    const int64_t b = blockIdx.x;
    const int t = threadIdx.x, lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
    Cube c;
    double a = 0.0, n = 0.0;
    if (cube_load(nbr + b * kNbr, u, emask, lx, ly, lz, c))
        cube_triangles(c, coords + 4 * b, lx, ly, lz, s, [&](const double *, const double *, const double *,
                                                             double ar) {
            a += ar;
            n += 1.0;
        });
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        n += __shfl_xor(n, o, 64);
    }
    if ((t & 63) == 0) { wa[t >> 6] = a; wn[t >> 6] = n; }
    __syncthreads();
    if (t == 0) {
        double sa = 0.0, sn = 0.0;
        for (int i = 0; i < 8; ++i) { sa += wa[i]; sn += wn[i]; }
        partials[2 * b] = sa;
        partials[2 * b + 1] = sn;
    }
}

__global__ void k_fill_zero_i64(int64_t *a) { *a = 0; }

__global__ void k_copy_coords(const int32_t *__restrict__ c4, int64_t nb, int32_t *__restrict__ out)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nb * 3) out[i] = c4[4 * (i / 3) + i % 3];
}

__global__ void k_unpack_keys(const uint64_t *__restrict__ k, int64_t n, int32_t *__restrict__ out)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t m = (uint64_t(1) << 21) - 1;
    const int64_t off = int64_t(1) << 20;
    out[3 * i] = int32_t(int64_t((k[i] >> 42) & m) - off);
    out[3 * i + 1] = int32_t(int64_t((k[i] >> 21) & m) - off);
    out[3 * i + 2] = int32_t(int64_t(k[i] & m) - off);
}

struct ScanScratch {
    int64_t *cnt, *ofs;
    void *tmp;
    size_t tmp_bytes;
};
static ScanScratch carve_scan(Bump &b, int64_t nb)
{
    ScanScratch x;
    x.cnt = b.take<int64_t>(size_t(nb) + 1);
    x.ofs = b.take<int64_t>(size_t(nb) + 1);
    x.tmp_bytes = tmp_light(size_t(nb) + 1);
    x.tmp = b.take<char>(x.tmp_bytes);
    return x;
}

size_t extract_scratch(int64_t n_blocks)
{
    Bump b(nullptr, 0);
    carve_scan(b, n_blocks);
    return b.off;
}

// Per-block counts (count_kernel) -> offsets -> total, in the scratch.
template <class CountK>
static int count_and_scan(dn_volume *v, CountK count_kernel, ScanScratch &x, int64_t *total)
{
    hipStream_t st = v->stream;
    const int64_t nb = v->nb;
    Bump bump(v->scratch, v->scratch_bytes);
    x = carve_scan(bump, nb);
    if (!bump.fits()) { set_error("scratch too small for the extraction"); return DN_E_CAPACITY; }
    if (nb > 0) {
        hipLaunchKernelGGL(count_kernel, dim3(unsigned(nb)), dim3(512), 0, st, nb, v->nbr, v->emask, v->u, x.cnt);
        DN_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_fill_zero_i64, dim3(1), dim3(1), 0, st, x.cnt + nb);
    DN_HIP(hipGetLastError());
    size_t tbytes = x.tmp_bytes;
    DN_HIP(rocprim::exclusive_scan(x.tmp, tbytes, x.cnt, x.ofs, int64_t(0), size_t(nb + 1), rocprim::plus<int64_t>(),
                                   st));
    int rc = read_back(v, x.ofs + nb, 8);
    if (rc) return rc;
    *total = v->host_stage[0];
    return DN_OK;
}

}  // namespace dn

using namespace dn;

extern "C" int dn_extract(dn_volume *v, int32_t what, void *out, size_t out_bytes, int64_t *n_out)
{
    DN_REQUIRE(v && n_out, "null argument");
    hipStream_t st = v->stream;
    const int64_t nb = v->nb, nv = nb * kBlockVox, ps = v->cap_blocks * kBlockVox;
    int64_t items = 0;
    size_t need = 0;
    int rc;
    uint64_t *uniq = nullptr;
    switch (what) {
    case DN_X_COORDS: items = nb; need = size_t(nb) * 12; break;
    case DN_X_HASH: items = v->hash_slots; need = size_t(items) * 16; break;
    case DN_X_NBR: items = nb; need = size_t(nb) * kNbr * 4; break;
    case DN_X_F: case DN_X_W: case DN_X_U: case DN_X_UBAR: items = nb; need = size_t(nv) * 4; break;
    case DN_X_P: items = nb; need = size_t(nv) * 12; break;
    case DN_X_EMASK: items = nb; need = size_t(nv); break;
    case DN_X_CANDIDATES:
        if ((rc = build_candidates(v, &uniq, &items))) return rc;
        need = size_t(items) * 12;
        break;
    case DN_X_SURFACE: {
        if ((rc = build_masks(v))) return rc;
        ScanScratch x;
        if ((rc = count_and_scan(v, k_surface_count, x, &items))) return rc;
        need = size_t(items) * 12;
        *n_out = items;
        if (items == 0) return DN_OK;
        if (!out || out_bytes < need) { set_error("output too small: need %zu bytes", need); return DN_E_CAPACITY; }
        hipLaunchKernelGGL(k_surface_write, dim3(unsigned(nb)), dim3(512), 0, st, nb, v->coords, v->nbr, v->emask,
                           v->u, x.ofs, v->prm.voxel_size, static_cast<float *>(out));
        DN_HIP(hipGetLastError());
        DN_HIP(hipStreamSynchronize(st));
        return DN_OK;
    }
    case DN_X_MESH: {
        if ((rc = build_masks(v))) return rc;
        ScanScratch x;
        if ((rc = count_and_scan(v, k_mesh_count, x, &items))) return rc;
        need = size_t(items) * 36;
        *n_out = items;
        if (items == 0) return DN_OK;
        if (!out || out_bytes < need) { set_error("output too small: need %zu bytes", need); return DN_E_CAPACITY; }
        hipLaunchKernelGGL(k_mesh_write, dim3(unsigned(nb)), dim3(512), 0, st, nb, v->coords, v->nbr, v->emask,
                           v->u, x.ofs, v->prm.voxel_size, static_cast<float *>(out));
        DN_HIP(hipGetLastError());
        DN_HIP(hipStreamSynchronize(st));
        return DN_OK;
    }
    default:
        set_error("unknown extract target %d", what);
        return DN_E_INVALID;
    }
    *n_out = items;
    if (need == 0) return DN_OK;
    if (!out || out_bytes < need) { set_error("output too small: need %zu bytes", need); return DN_E_CAPACITY; }
    switch (what) {
    case DN_X_COORDS:
        hipLaunchKernelGGL(k_copy_coords, dim3(grid1(nb * 3)), dim3(256), 0, st, v->coords, nb, static_cast<int32_t *>(out));
        DN_HIP(hipGetLastError());
        break;
    case DN_X_HASH: DN_HIP(hipMemcpyAsync(out, v->hash[v->cur_hash], need, hipMemcpyDeviceToDevice, st)); break;
    case DN_X_NBR: DN_HIP(hipMemcpyAsync(out, v->nbr, need, hipMemcpyDeviceToDevice, st)); break;
    case DN_X_F: DN_HIP(hipMemcpyAsync(out, v->f, need, hipMemcpyDeviceToDevice, st)); break;
    case DN_X_W: DN_HIP(hipMemcpyAsync(out, v->w, need, hipMemcpyDeviceToDevice, st)); break;
    case DN_X_U: DN_HIP(hipMemcpyAsync(out, v->u, need, hipMemcpyDeviceToDevice, st)); break;
    case DN_X_UBAR: DN_HIP(hipMemcpyAsync(out, v->ubar[v->cur], need, hipMemcpyDeviceToDevice, st)); break;
    case DN_X_P:
        for (int a = 0; a < 3; ++a)
            DN_HIP(hipMemcpyAsync(static_cast<float *>(out) + a * nv, v->p[v->cur] + a * ps, size_t(nv) * 4,
                                  hipMemcpyDeviceToDevice, st));
        break;
    case DN_X_EMASK:
        if ((rc = build_masks(v))) return rc;
        DN_HIP(hipMemcpyAsync(out, v->emask, need, hipMemcpyDeviceToDevice, st));
        break;
    case DN_X_CANDIDATES:
        hipLaunchKernelGGL(k_unpack_keys, dim3(grid1(items)), dim3(256), 0, st, uniq, items,
                           static_cast<int32_t *>(out));
        DN_HIP(hipGetLastError());
        break;
    }
    DN_HIP(hipStreamSynchronize(st));
    return DN_OK;
}

// Total area (float64) and number of the mesh's triangles.
extern "C" int dn_mesh_area(dn_volume *v, double *area, int64_t *n_tris)
{
    DN_REQUIRE(v && area, "null argument");
    int rc;
    if ((rc = build_masks(v))) return rc;
    double ed[2] = {0.0, 0.0};
    if (v->nb > 0) {
        hipLaunchKernelGGL(k_mesh_area, dim3(unsigned(v->nb)), dim3(512), 0, v->stream, v->nb, v->coords, v->nbr,
                           v->emask, v->u, v->prm.voxel_size, v->partials);
        DN_HIP(hipGetLastError());
        if ((rc = reduce_pairs(v, v->nb))) return rc;
        if ((rc = read_energy(v, ed))) return rc;
    }
    *area = ed[0];
    if (n_tris) *n_tris = int64_t(ed[1]);
    return DN_OK;
}
