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
    switch (what) {
    case DN_X_COORDS: items = nb; need = size_t(nb) * 12; break;
    case DN_X_HASH: items = v->hash_slots; need = size_t(items) * 16; break;
    case DN_X_NBR: items = nb; need = size_t(nb) * kNbr * 4; break;
    case DN_X_F: case DN_X_W: case DN_X_U: case DN_X_UBAR: items = nb; need = size_t(nv) * 4; break;
    case DN_X_P: items = nb; need = size_t(nv) * 12; break;
    case DN_X_EMASK: items = nb; need = size_t(nv); break;
    case DN_X_CANDIDATES: items = v->last_nuniq; need = size_t(items) * 12; break;
    case DN_X_SURFACE: {
        if ((rc = build_masks(v))) return rc;
        if ((rc = v->s_counts.ensure((nb + 1) * 8))) return rc;
        if ((rc = v->s_offsets.ensure((nb + 1) * 8))) return rc;
        int64_t *cnt = v->s_counts.as<int64_t>(), *ofs = v->s_offsets.as<int64_t>();
        if (nb > 0) {
            hipLaunchKernelGGL(k_surface_count, dim3(unsigned(nb)), dim3(512), 0, st, nb, v->nbr, v->emask, v->u, cnt);
            DN_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_fill_zero_i64, dim3(1), dim3(1), 0, st, cnt + nb);
        DN_HIP(hipGetLastError());
        size_t tb = 0;
        DN_HIP(rocprim::exclusive_scan(nullptr, tb, cnt, ofs, int64_t(0), size_t(nb + 1), rocprim::plus<int64_t>(), st));
        if ((rc = v->s_tmp.ensure(tb))) return rc;
        size_t tbytes = v->s_tmp.bytes;
        DN_HIP(rocprim::exclusive_scan(v->s_tmp.ptr, tbytes, cnt, ofs, int64_t(0), size_t(nb + 1),
                                       rocprim::plus<int64_t>(), st));
        if ((rc = v->host.ensure(64))) return rc;
        DN_HIP(hipMemcpyAsync(v->host.ptr, ofs + nb, 8, hipMemcpyDeviceToHost, st));
        DN_HIP(hipStreamSynchronize(st));
        items = v->host.as<int64_t>()[0];
        need = size_t(items) * 12;
        *n_out = items;
        if (items == 0) return DN_OK;
        if (!out || out_bytes < need) { set_error("output too small: need %zu bytes", need); return DN_E_CAPACITY; }
        hipLaunchKernelGGL(k_surface_write, dim3(unsigned(nb)), dim3(512), 0, st, nb, v->coords, v->nbr, v->emask,
                           v->u, ofs, v->prm.voxel_size, static_cast<float *>(out));
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
        hipLaunchKernelGGL(k_unpack_keys, dim3(grid1(items)), dim3(256), 0, st, v->s_uniq.as<uint64_t>(), items,
                           static_cast<int32_t *>(out));
        DN_HIP(hipGetLastError());
        break;
    }
    DN_HIP(hipStreamSynchronize(st));
    return DN_OK;
}
