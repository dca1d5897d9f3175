// Omega-masked TV primal-dual regulariser over hashed 8^3 blocks (gfx950).
//
// Section III-B/C of the paper: masked forward-difference gradient (Eq. 3),
// its negative adjoint as divergence (Eq. 4), and the Chambolle-Pock
// iteration (Eqs. 7-9) on the weighted ROF energy.  Two implementations of
// one iteration:
//   - two-pass: a dual kernel and a primal kernel, in place (60 B/voxel);
//   - fused: one kernel per iteration; each workgroup stages its block's
//     ubar with a one-voxel halo in LDS, recomputes the new dual on the -1
//     halo faces (so no second pass is needed) and ping-pongs ubar and p
//     between two buffers (48 B/voxel of algorithmic traffic).
// The fused body is shared with a persistent kernel that runs many
// sub-maps and all iterations in one launch, separated by grid barriers.
// Energies are accumulated in float64 with a fixed reduction order.
#include <cstring>
#include <rocprim/rocprim.hpp>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "cp_kernel.h"
#include "dn_internal.h"

namespace dn {

template <class S, bool kRefine>
__global__ __launch_bounds__(512) void k_cp_fused(CPArgs<S> A)
{
    __shared__ CPShared sh;
    int64_t slot = block_slot(blockIdx.x, A.nb, A.xcd);
    if (slot >= A.nb) return;
    int64_t b = A.order ? A.order[slot] : slot;
    cp_block<S, kRefine, 512>(A, b, sh, threadIdx.x);
}

// The same iteration with 256 threads per block (two voxels per thread):
// twice the loads in flight per thread and twice the workgroups per CU.
template <class S, bool kRefine>
__global__ __launch_bounds__(256) void k_cp_fused256(CPArgs<S> A)
{
    __shared__ CPShared sh;
    int64_t slot = block_slot(blockIdx.x, A.nb, A.xcd);
    if (slot >= A.nb) return;
    int64_t b = A.order ? A.order[slot] : slot;
    cp_block<S, kRefine, 256>(A, b, sh, threadIdx.x);
}

// ----------------------------------------------------- two-pass variant
__global__ __launch_bounds__(512) void k_dual(int64_t nb, int64_t ps, const int32_t *__restrict__ nbr,
                                              const uint8_t *__restrict__ emask, const float *__restrict__ ubar,
                                              float *__restrict__ p, float sigma)
{
    const int64_t b = blockIdx.x;
    if (b >= nb) return;
    const int t = threadIdx.x, lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
    const int64_t gi = b * kBlockVox + t;
    const int32_t *nb27 = nbr + b * kNbr;
    const uint8_t m = emask[gi];
    const float u0 = ubar[gi];
    float g[3] = {0.f, 0.f, 0.f};
    if (m & 2) g[0] = ubar[lx < 7 ? gi + 1 : halo_index(nb27, 8, ly, lz)] - u0;
    if (m & 4) g[1] = ubar[ly < 7 ? gi + 8 : halo_index(nb27, lx, 8, lz)] - u0;
    if (m & 8) g[2] = ubar[lz < 7 ? gi + 64 : halo_index(nb27, lx, ly, 8)] - u0;
    float a = p[gi] + sigma * g[0], c1 = p[gi + ps] + sigma * g[1], c2 = p[gi + 2 * ps] + sigma * g[2];
    project(a, c1, c2);
    p[gi] = a; p[gi + ps] = c1; p[gi + 2 * ps] = c2;
}

__global__ __launch_bounds__(512) void k_primal(int64_t nb, int64_t ps, const int32_t *__restrict__ nbr,
                                                const uint8_t *__restrict__ emask, const float *__restrict__ p,
                                                const float *__restrict__ f, const float *__restrict__ w,
                                                float *__restrict__ u, float *__restrict__ ubar, float tau,
                                                float lambda, float theta, int l1)
{
    const int64_t b = blockIdx.x;
    if (b >= nb) return;
    const int t = threadIdx.x, lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
    const int64_t gi = b * kBlockVox + t;
    const int32_t *nb27 = nbr + b * kNbr;
    const uint8_t m = emask[gi];
    const float uo = u[gi];
    float un = uo;
    if (m & 1) {
        float dv = 0.0f;
        for (int a = 0; a < 3; ++a) {
            int64_t jm;
            if (a == 0) jm = lx > 0 ? gi - 1 : halo_index(nb27, -1, ly, lz);
            else if (a == 1) jm = ly > 0 ? gi - 8 : halo_index(nb27, lx, -1, lz);
            else jm = lz > 0 ? gi - 64 : halo_index(nb27, lx, ly, -1);
            const uint8_t bit = uint8_t(2 << a);
            float fwd = (m & bit) ? p[gi + a * ps] : 0.0f;
            float bwd = (jm >= 0 && (emask[jm] & bit)) ? p[jm + a * ps] : 0.0f;
            dv += fwd - bwd;
        }
        float ut = uo + tau * dv;
        float tlw = tau * lambda * w[gi];
        if (l1) {
            float r = ut - f[gi];
            r = r > tlw ? r - tlw : (r < -tlw ? r + tlw : 0.0f);
            un = fminf(fmaxf(f[gi] + r, -1.0f), 1.0f);
        } else {
            un = (ut + tlw * f[gi]) / (1.0f + tlw);
        }
    }
    u[gi] = un;
    ubar[gi] = un + theta * (un - uo);
}

// ------------------------------------------------------------- masks
// emask bit0 = Omega(g) (block allocated and w > 0); bit 1+a = m_a(g) =
// Omega(g) and Omega(g + e_a)  (Eq. 3's cases where the difference is kept).
__global__ __launch_bounds__(512) void k_masks(int64_t nb, const int32_t *__restrict__ nbr,
                                               const float *__restrict__ w, uint8_t *__restrict__ emask)
{
    const int64_t b = blockIdx.x;
    if (b >= nb) return;
    const int t = threadIdx.x, lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
    const int64_t gi = b * kBlockVox + t;
    const int32_t *nb27 = nbr + b * kNbr;
    uint8_t m = 0;
    if (w[gi] > 0.0f) {
        m = 1;
        int64_t jx = halo_index(nb27, lx + 1, ly, lz);
        int64_t jy = halo_index(nb27, lx, ly + 1, lz);
        int64_t jz = halo_index(nb27, lx, ly, lz + 1);
        if (jx >= 0 && w[jx] > 0.0f) m |= 2;
        if (jy >= 0 && w[jy] > 0.0f) m |= 4;
        if (jz >= 0 && w[jz] > 0.0f) m |= 8;
    }
    emask[gi] = m;
}

__device__ __forceinline__ uint64_t spread3(uint64_t v)
{
    v &= 0x1FFFFF;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__global__ void k_morton(const int32_t *__restrict__ coords, int64_t nb, uint64_t *__restrict__ code,
                         int32_t *__restrict__ ids)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    uint64_t x = uint64_t(int64_t(coords[4 * i]) + (1 << 20));
    uint64_t y = uint64_t(int64_t(coords[4 * i + 1]) + (1 << 20));
    uint64_t z = uint64_t(int64_t(coords[4 * i + 2]) + (1 << 20));
    code[i] = spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
    ids[i] = int32_t(i);
}

// ---------------------------------------------------------- energies
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Per-block partial sums of E(u) and D(p) (Eq. 2 with the weight of the
// proximal step, Eq. 6), float64.  256 threads, two voxels each; u with its
// +1 faces, p and the edge masks with their -1 faces are staged in LDS.
// Fixed reduction order: lanes by xor-shuffle butterflies, then the 4 wave
// sums in wave order.
template <class S>
__global__ __launch_bounds__(256) void k_energy_partial(int64_t nb, int64_t ps, const int32_t *__restrict__ nbr,
                                                        const uint8_t *__restrict__ emask,
                                                        const typename S::T *__restrict__ u,
                                                        const typename S::T *__restrict__ p,
                                                        const float *__restrict__ f, const float *__restrict__ w,
                                                        double lambda, int l1, double *__restrict__ partials)
{
    __shared__ float su[729];        // u on [0, 8]^3, index ((z*9)+y)*9+x
    __shared__ float sp[3][729];     // p on [-1, 7]^3, index i9
    __shared__ uint8_t sm[729];      // edge masks on [-1, 7]^3, index i9
    __shared__ double se[4], sd[4];
    const int64_t b = blockIdx.x;
    if (b >= nb) return;
    const int t = threadIdx.x;
    const int32_t *nb27 = nbr + b * kNbr;
    auto iu = [](int x, int y, int z) { return (z * 9 + y) * 9 + x; };
    for (int k = 0; k < 2; ++k) {
        const int v = t + 256 * k, lx = v & 7, ly = (v >> 3) & 7, lz = v >> 6;
        const int64_t gi = b * kBlockVox + v;
        su[iu(lx, ly, lz)] = S::ld(u[gi]);
        const int q = i9(lx, ly, lz);
        sm[q] = emask[gi];
        sp[0][q] = S::ld(p[gi]); sp[1][q] = S::ld(p[gi + ps]); sp[2][q] = S::ld(p[gi + 2 * ps]);
    }
    if (t < 192) {
        // +1 faces of u: face a = t / 64
        const int a = t >> 6, i = t & 63, c0 = i & 7, c1 = i >> 3;
        int x, y, z;
        if (a == 0) { x = 8; y = c0; z = c1; }
        else if (a == 1) { x = c0; y = 8; z = c1; }
        else { x = c0; y = c1; z = 8; }
        int64_t j = halo_index(nb27, x, y, z);
        su[iu(x, y, z)] = j >= 0 ? S::ld(u[j]) : 0.0f;
        // -1 faces: the normal component of p and the edge mask
        int hx, hy, hz;
        face_pos(t, hx, hy, hz);
        int64_t jm = halo_index(nb27, hx, hy, hz);
        const int q = i9(hx, hy, hz);
        sm[q] = jm >= 0 ? emask[jm] : uint8_t(0);
        sp[a][q] = jm >= 0 ? S::ld(p[jm + a * ps]) : 0.0f;
    }
    __syncthreads();
    double e = 0.0, d = 0.0;
    for (int k = 0; k < 2; ++k) {
        const int v = t + 256 * k, lx = v & 7, ly = (v >> 3) & 7, lz = v >> 6;
        const int q = i9(lx, ly, lz);
        const uint8_t m = sm[q];
        if (!(m & 1)) continue;
        const int64_t gi = b * kBlockVox + v;
        const double u0 = su[iu(lx, ly, lz)];
        const double g0 = (m & 2) ? double(su[iu(lx + 1, ly, lz)]) - u0 : 0.0;
        const double g1 = (m & 4) ? double(su[iu(lx, ly + 1, lz)]) - u0 : 0.0;
        const double g2 = (m & 8) ? double(su[iu(lx, ly, lz + 1)]) - u0 : 0.0;
        const double fv = f[gi], wv = w[gi];
        const double r = u0 - fv;
        e += sqrt((g0 * g0 + g1 * g1) + g2 * g2) + (l1 ? lambda * wv * fabs(r) : 0.5 * lambda * wv * r * r);
        const int qx = i9(lx - 1, ly, lz), qy = i9(lx, ly - 1, lz), qz = i9(lx, ly, lz - 1);
        double dv = 0.0;
        dv += ((m & 2) ? double(sp[0][q]) : 0.0) - ((sm[qx] & 2) ? double(sp[0][qx]) : 0.0);
        dv += ((m & 4) ? double(sp[1][q]) : 0.0) - ((sm[qy] & 4) ? double(sp[1][qy]) : 0.0);
        dv += ((m & 8) ? double(sp[2][q]) : 0.0) - ((sm[qz] & 8) ? double(sp[2][qz]) : 0.0);
        if (l1) {
            // minimum over u in [-1, 1] of -u d + lambda w |u - f|: at -1, f or 1
            const double lw = lambda * wv;
            const double c0 = -fv * dv, c1 = -dv + lw * fabs(1.0 - fv), c2 = dv + lw * fabs(1.0 + fv);
            d += fmin(fmin(c0, c1), c2);
        } else {
            d += -fv * dv - dv * dv / (2.0 * lambda * wv);
        }
    }
    e = wave_sum(e);
    d = wave_sum(d);
    const int wave = t >> 6;
    if ((t & 63) == 0) { se[wave] = e; sd[wave] = d; }
    __syncthreads();
    if (t == 0) {
        partials[2 * b] = ((se[0] + se[1]) + se[2]) + se[3];
        partials[2 * b + 1] = ((sd[0] + sd[1]) + sd[2]) + sd[3];
    }
}

// Fixed-order reduction of n (E, D) pairs: workgroup g sums pairs
// [1024 g, 1024 g + 1024): each thread adds 4 consecutive pairs, then a
// tree over the 256 threads.
__global__ __launch_bounds__(256) void k_energy_reduce(int64_t n, const double *__restrict__ in,
                                                       double *__restrict__ out)
{
    __shared__ double se[256], sd[256];
    const int t = threadIdx.x;
    const int64_t base = int64_t(blockIdx.x) * 1024 + 4 * t;
    double e = 0.0, d = 0.0;
    for (int k = 0; k < 4; ++k)
        if (base + k < n) { e += in[2 * (base + k)]; d += in[2 * (base + k) + 1]; }
    se[t] = e; sd[t] = d;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) { se[t] += se[t + h]; sd[t] += sd[t + h]; }
        __syncthreads();
    }
    if (t == 0) { out[2 * blockIdx.x] = se[0]; out[2 * blockIdx.x + 1] = sd[0]; }
}

// ------------------------------------------------------- helpers
template <class T> __global__ void k_fill(T *__restrict__ a, int64_t n, T v)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

template <class S> __global__ void k_demote(const float *__restrict__ a, typename S::T *__restrict__ b, int64_t n, int rz)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) b[i] = rz ? S::rz(a[i]) : S::rn(a[i]);
}

template <class S> __global__ void k_promote(const typename S::T *__restrict__ b, float *__restrict__ a, int64_t n)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) a[i] = S::ld(b[i]);
}

static inline unsigned grid1(int64_t n, int bs = 256) { return unsigned((n + bs - 1) / bs); }

template <class T> static int fill(hipStream_t st, T *a, int64_t n, T v)
{
    if (n <= 0) return DN_OK;
    hipLaunchKernelGGL(k_fill<T>, dim3(grid1(n)), dim3(256), 0, st, a, n, v);
    DN_HIP(hipGetLastError());
    return DN_OK;
}

struct MaskScratch {
    uint64_t *code, *code2;
    int32_t *ids;
    void *tmp;
    size_t tmp_bytes;
};
static MaskScratch carve_masks(Bump &b, int64_t nb)
{
    MaskScratch x;
    x.code = b.take<uint64_t>(size_t(nb));
    x.code2 = b.take<uint64_t>(size_t(nb));
    x.ids = b.take<int32_t>(size_t(nb));
    x.tmp_bytes = tmp_sort(size_t(nb), 12);
    x.tmp = b.take<char>(x.tmp_bytes);
    return x;
}

size_t masks_scratch(int64_t n_blocks)
{
    Bump b(nullptr, 0);
    carve_masks(b, n_blocks);
    return b.off;
}

int build_masks(dn_volume *v)
{
    if (v->emask_nb == v->nb) return DN_OK;
    hipStream_t st = v->stream;
    if (v->nb > 0) {
        hipLaunchKernelGGL(k_masks, dim3(unsigned(v->nb)), dim3(512), 0, st, v->nb, v->nbr, v->w, v->emask);
        DN_HIP(hipGetLastError());
        // Morton processing order of the blocks
        Bump bump(v->scratch, v->scratch_bytes);
        MaskScratch x = carve_masks(bump, v->nb);
        if (!bump.fits()) { set_error("scratch too small for the block order"); return DN_E_CAPACITY; }
        hipLaunchKernelGGL(k_morton, dim3(grid1(v->nb)), dim3(256), 0, st, v->coords, v->nb, x.code, x.ids);
        DN_HIP(hipGetLastError());
        size_t tbytes = x.tmp_bytes;
        DN_HIP(rocprim::radix_sort_pairs(x.tmp, tbytes, x.code, x.code2, x.ids, v->order, size_t(v->nb), 0, 63, st));
    }
    v->emask_nb = v->nb;
    return DN_OK;
}

template <class S>
static int energy_launch(dn_volume *v, double lambda, int l1, const typename S::T *u, const typename S::T *p)
{
    hipStream_t st = v->stream;
    const int64_t ps = v->cap_blocks * kBlockVox;
    if (v->nb == 0) {
        hipLaunchKernelGGL(k_fill<double>, dim3(1), dim3(256), 0, st, v->energy2, int64_t(2), 0.0);
        DN_HIP(hipGetLastError());
        return DN_OK;
    }
    hipLaunchKernelGGL((k_energy_partial<S>), dim3(unsigned(v->nb)), dim3(256), 0, st, v->nb, ps, v->nbr,
                       v->emask, u, p, v->f, v->w, lambda, l1, v->partials);
    DN_HIP(hipGetLastError());
    return reduce_pairs(v, v->nb);
}

// Fixed-order sum of the n per-block pairs in v->partials into
// v->energy2: level by level (ping-pong inside the scratch that follows the
// per-block partials) until one pair is left.
int reduce_pairs(dn_volume *v, int64_t n)
{
    hipStream_t st = v->stream;
    double *src = v->partials;
    double *bufs[2] = {v->partials + 2 * v->cap_blocks, v->partials + 2 * v->cap_blocks + 2 * ((v->cap_blocks + 1023) / 1024 + 1)};
    int which = 0;
    while (n > 1) {
        const int64_t g = (n + 1023) / 1024;
        double *dst = (g == 1) ? v->energy2 : bufs[which];
        hipLaunchKernelGGL(k_energy_reduce, dim3(unsigned(g)), dim3(256), 0, st, n, src, dst);
        DN_HIP(hipGetLastError());
        src = dst;
        which ^= 1;
        n = g;
    }
    if (src != v->energy2) DN_HIP(hipMemcpyAsync(v->energy2, src, 16, hipMemcpyDeviceToDevice, st));
    return DN_OK;
}

// Energies of the current state into v->energy2 (device).
int energy_current(dn_volume *v, double lambda, bool use_f32, int data_term)
{
    const int l1 = data_term == DN_DATA_L1;
    int rc = build_masks(v);
    if (rc) return rc;
    switch (use_f32 ? DN_F32 : v->state_storage) {
    case DN_F16:
        return energy_launch<SF16>(v, lambda, l1, (const uint16_t *)v->u16, (const uint16_t *)v->p16[v->cur]);
    case DN_BF16:
        return energy_launch<SBF16>(v, lambda, l1, (const uint16_t *)v->u16, (const uint16_t *)v->p16[v->cur]);
    default:
        return energy_launch<SF32>(v, lambda, l1, v->u, v->p[v->cur]);
    }
}

int read_energy(dn_volume *v, double out[2])
{
    int rc = read_back(v, v->energy2, 16);
    if (rc) return rc;
    memcpy(out, v->host_stage, 16);
    return DN_OK;
}

template <class S>
static CPArgs<S> make_args(dn_volume *v, const dn_reg_params *prm, typename S::T *u, typename S::T *ub_in,
                           typename S::T *ub_out, typename S::T *p_in, typename S::T *p_out)
{
    CPArgs<S> A;
    A.nb = v->nb;
    A.pstride = v->cap_blocks * kBlockVox;
    A.nbr = v->nbr;
    A.emask = v->emask;
    A.order = v->layout & 1 ? nullptr : v->order;
    A.xcd = (v->layout & 2) ? 0 : 1;
    A.f = v->f; A.w = v->w;
    A.u = u; A.ubar_in = ub_in; A.ubar_out = ub_out; A.p_in = p_in; A.p_out = p_out;
    A.u32 = nullptr; A.ubar32 = nullptr; A.p32 = nullptr;
    A.sigma = float(prm->sigma); A.tau = float(prm->tau); A.lambda = float(prm->lambda);
    A.theta = float(prm->theta);
    A.l1 = prm->data_term == DN_DATA_L1;
    A.seed = 0u;
    return A;
}

static unsigned fused_grid(int64_t nb) { return unsigned(((nb + 7) / 8) * 8); }

// One FP32 iteration with the chosen kernel.
static int step_f32(dn_volume *v, const dn_reg_params *prm, int kernel)
{
    hipStream_t st = v->stream;
    const int64_t ps = v->cap_blocks * kBlockVox;
    if (kernel == DN_K_TWOPASS) {
        hipLaunchKernelGGL(k_dual, dim3(unsigned(v->nb)), dim3(512), 0, st, v->nb, ps, v->nbr, v->emask,
                           v->ubar[v->cur], v->p[v->cur], float(prm->sigma));
        DN_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_primal, dim3(unsigned(v->nb)), dim3(512), 0, st, v->nb, ps, v->nbr, v->emask,
                           v->p[v->cur], v->f, v->w, v->u, v->ubar[v->cur], float(prm->tau), float(prm->lambda),
                           float(prm->theta), int(prm->data_term == DN_DATA_L1));
        DN_HIP(hipGetLastError());
        return DN_OK;
    }
    const int c = v->cur, n = 1 - c;
    auto A = make_args<SF32>(v, prm, v->u, v->ubar[c], v->ubar[n], v->p[c], v->p[n]);
    if (kernel == DN_K_FUSED256)
        hipLaunchKernelGGL((k_cp_fused256<SF32, false>), dim3(fused_grid(v->nb)), dim3(256), 0, st, A);
    else
        hipLaunchKernelGGL((k_cp_fused<SF32, false>), dim3(fused_grid(v->nb)), dim3(512), 0, st, A);
    DN_HIP(hipGetLastError());
    v->cur = n;
    return DN_OK;
}

template <class S>
static int step_lowp(dn_volume *v, const dn_reg_params *prm, bool refine, int kernel)
{
    const int c = v->cur, n = 1 - c;
    using T = typename S::T;
    auto A = make_args<S>(v, prm, (T *)v->u16, (T *)v->ubar16[c], (T *)v->ubar16[n], (T *)v->p16[c],
                          (T *)v->p16[n]);
    A.seed = uint32_t(v->lowp_iter++);
    const dim3 grid(fused_grid(v->nb));
    if (refine) {
        A.u32 = v->u; A.ubar32 = v->ubar[n]; A.p32 = v->p[n];
        if (kernel == DN_K_FUSED256)
            hipLaunchKernelGGL((k_cp_fused256<S, true>), grid, dim3(256), 0, v->stream, A);
        else
            hipLaunchKernelGGL((k_cp_fused<S, true>), grid, dim3(512), 0, v->stream, A);
    } else {
        if (kernel == DN_K_FUSED256)
            hipLaunchKernelGGL((k_cp_fused256<S, false>), grid, dim3(256), 0, v->stream, A);
        else
            hipLaunchKernelGGL((k_cp_fused<S, false>), grid, dim3(512), 0, v->stream, A);
    }
    DN_HIP(hipGetLastError());
    v->cur = n;
    return DN_OK;
}

// Copy the FP32 state into the 16-bit buffers (u, ubar round to nearest,
// p toward zero so |p| <= 1 survives the rounding).
template <class S> static int demote_state(dn_volume *v)
{
    hipStream_t st = v->stream;
    const int64_t n = v->nb * kBlockVox, ps = v->cap_blocks * kBlockVox;
    using T = typename S::T;
    if (n == 0) return DN_OK;
    hipLaunchKernelGGL((k_demote<S>), dim3(grid1(n)), dim3(256), 0, st, v->u, (T *)v->u16, n, 0);
    hipLaunchKernelGGL((k_demote<S>), dim3(grid1(n)), dim3(256), 0, st, v->ubar[v->cur], (T *)v->ubar16[v->cur], n, 0);
    for (int a = 0; a < 3; ++a)
        hipLaunchKernelGGL((k_demote<S>), dim3(grid1(n)), dim3(256), 0, st, v->p[v->cur] + a * ps,
                           (T *)v->p16[v->cur] + a * ps, n, 1);
    DN_HIP(hipGetLastError());
    return DN_OK;
}

static int validate(const dn_reg_params *prm)
{
    DN_REQUIRE(prm, "null params");
    DN_REQUIRE(prm->lambda > 0 && prm->tau > 0 && prm->sigma > 0, "lambda, tau, sigma must be > 0");
    DN_REQUIRE(prm->tau * prm->sigma * 12.0 <= 1.0 + 1e-9,
               "step sizes violate tau*sigma*|grad|^2 <= 1 (|grad|^2 <= 12 in 3-D)");
    DN_REQUIRE(prm->theta >= 0 && prm->theta <= 1, "theta must be in [0, 1]");
    DN_REQUIRE(prm->iters >= 0 && prm->gap_every >= 0, "iters, gap_every must be >= 0");
    int s = prm->storage;
    DN_REQUIRE(s == DN_F32 || s == DN_F16 || s == DN_BF16, "bad storage");
    DN_REQUIRE(prm->init >= DN_INIT_ZERO && prm->init <= DN_INIT_CONTINUE, "bad init");
    DN_REQUIRE(prm->kernel >= DN_K_AUTO && prm->kernel <= DN_K_FUSED256, "bad kernel");
    DN_REQUIRE(prm->refine_every >= 0, "refine_every must be >= 0");
    DN_REQUIRE(prm->gamma >= 0 && std::isfinite(prm->gamma), "gamma must be >= 0");
    DN_REQUIRE(prm->data_term == DN_DATA_L2 || prm->data_term == DN_DATA_L1, "bad data_term");
    DN_REQUIRE(prm->data_term == DN_DATA_L2 || prm->gamma == 0.0,
               "the accelerated variant needs the uniformly convex (L2) data term");
    return DN_OK;
}

// Copy the 16-bit state (exactly) into the FP32 buffers, so that a 16-bit
// run that stopped between refinement sweeps leaves its current state
// where the extraction and an FP32 continuation read it.
template <class S> static int promote_state(dn_volume *v)
{
    hipStream_t st = v->stream;
    const int64_t n = v->nb * kBlockVox, ps = v->cap_blocks * kBlockVox;
    using T = typename S::T;
    if (n == 0) return DN_OK;
    hipLaunchKernelGGL((k_promote<S>), dim3(grid1(n)), dim3(256), 0, st, (const T *)v->u16, v->u, n);
    hipLaunchKernelGGL((k_promote<S>), dim3(grid1(n)), dim3(256), 0, st, (const T *)v->ubar16[v->cur],
                       v->ubar[v->cur], n);
    for (int a = 0; a < 3; ++a)
        hipLaunchKernelGGL((k_promote<S>), dim3(grid1(n)), dim3(256), 0, st, (const T *)v->p16[v->cur] + a * ps,
                           v->p[v->cur] + a * ps, n);
    DN_HIP(hipGetLastError());
    return DN_OK;
}

int zero_state(dn_volume *v)
{
    hipStream_t st = v->stream;
    const int64_t n = v->nb * kBlockVox, ps = v->cap_blocks * kBlockVox;
    int rc;
    if ((rc = fill<float>(st, v->u, n, 0.f))) return rc;
    if ((rc = fill<float>(st, v->ubar[v->cur], n, 0.f))) return rc;
    for (int a = 0; a < 3; ++a)
        if ((rc = fill<float>(st, v->p[v->cur] + a * ps, n, 0.f))) return rc;
    v->state_storage = DN_F32;
    return DN_OK;
}

// Kernel choice for DN_K_AUTO: measured once per size bucket.  A choice is
// (kernel variant, layout) with layout bit 0 = pool order instead of Morton
// order, bit 1 = plain workgroup -> block map instead of XCD chunks.
struct AutoChoice { int kernel; int layout; };
// Keyed by (device, size bucket); the tuners of all threads share them.
static std::map<int64_t, AutoChoice> g_auto_kernel;
static std::mutex g_auto_mutex;

static int size_bucket(int64_t nb)
{
    int b = 0;
    while ((int64_t(1) << b) < nb) ++b;
    return b;
}

static int64_t tune_key(const dn_volume *v, int64_t sub) { return (int64_t(v->device) << 32) | sub; }

static bool find_choice(std::map<int64_t, AutoChoice> &m, int64_t key, AutoChoice *out)
{
    std::lock_guard<std::mutex> lk(g_auto_mutex);
    auto it = m.find(key);
    if (it == m.end()) return false;
    *out = it->second;
    return true;
}

static void store_choice(std::map<int64_t, AutoChoice> &m, int64_t key, AutoChoice c)
{
    std::lock_guard<std::mutex> lk(g_auto_mutex);
    m[key] = c;
}

static int autotune_single(dn_volume *v, const dn_reg_params *prm, int *choice)
{
    const int64_t key = tune_key(v, size_bucket(v->nb));
    AutoChoice found;
    if (find_choice(g_auto_kernel, key, &found)) {
        *choice = found.kernel;
        v->layout = found.layout;
        return DN_OK;
    }
    // time a few iterations of each candidate from the zero state
    hipEvent_t e0, e1;
    DN_HIP(hipEventCreate(&e0));
    DN_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    AutoChoice best{DN_K_FUSED, 0};
    const int trial = 6;
    for (int k : {DN_K_TWOPASS, DN_K_FUSED, DN_K_FUSED256})
        for (int layout = 0; layout < 4; ++layout) {
            if (k == DN_K_TWOPASS && layout != 0) continue;   // the two-pass kernels use pool order
            v->layout = layout;
            int rc = zero_state(v);
            if (rc) return rc;
            if ((rc = step_f32(v, prm, k))) return rc;  // warm up
            DN_HIP(hipEventRecord(e0, v->stream));
            for (int i = 0; i < trial; ++i)
                if ((rc = step_f32(v, prm, k))) return rc;
            DN_HIP(hipEventRecord(e1, v->stream));
            DN_HIP(hipEventSynchronize(e1));
            float ms = 0;
            DN_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (getenv("DN_VERBOSE"))
                fprintf(stderr, "[denser] tune: kernel %d layout %d: %.4f ms per iteration\n", k, layout, ms / trial);
            if (ms < best_ms) { best_ms = ms; best = AutoChoice{k, layout}; }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    store_choice(g_auto_kernel, key, best);
    *choice = best.kernel;
    v->layout = best.layout;
    return zero_state(v);
}

// The same choice for 16-bit state storage, timed on the 16-bit kernels.
// It runs only on a state just demoted from FP32 (the trials overwrite the
// 16-bit buffers, which are then demoted again).
static std::map<int64_t, AutoChoice> g_auto_lowp;

template <class S> static int autotune_lowp(dn_volume *v, const dn_reg_params *prm, int storage, int *choice)
{
    const int64_t key = tune_key(v, storage * 64 + size_bucket(v->nb));
    AutoChoice found;
    if (find_choice(g_auto_lowp, key, &found)) {
        *choice = found.kernel;
        v->layout = found.layout;
        return DN_OK;
    }
    hipEvent_t e0, e1;
    DN_HIP(hipEventCreate(&e0));
    DN_HIP(hipEventCreate(&e1));
    const int cur = v->cur;
    const uint64_t seed_iter = v->lowp_iter;   // the trials are discarded, so are their seeds
    float best_ms = 1e30f;
    AutoChoice best{DN_K_FUSED, 0};
    const int trial = 6;
    int rc = DN_OK;
    for (int k : {DN_K_FUSED, DN_K_FUSED256})
        for (int layout = 0; layout < 4 && !rc; ++layout) {
            v->layout = layout;
            if ((rc = step_lowp<S>(v, prm, false, k))) break;   // warm up
            DN_HIP(hipEventRecord(e0, v->stream));
            for (int i = 0; i < trial && !rc; ++i) rc = step_lowp<S>(v, prm, false, k);
            DN_HIP(hipEventRecord(e1, v->stream));
            DN_HIP(hipEventSynchronize(e1));
            float ms = 0;
            DN_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (getenv("DN_VERBOSE"))
                fprintf(stderr, "[denser] tune16: kernel %d layout %d: %.4f ms per iteration\n", k, layout, ms / trial);
            if (ms < best_ms) { best_ms = ms; best = AutoChoice{k, layout}; }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    v->cur = cur;
    v->lowp_iter = seed_iter;
    if (rc) return rc;
    store_choice(g_auto_lowp, key, best);
    *choice = best.kernel;
    v->layout = best.layout;
    return demote_state<S>(v);
}

}  // namespace dn

using namespace dn;

extern "C" {

int dn_energy(dn_volume *v, double lambda, int32_t data_term, double out[2])
{
    DN_REQUIRE(v && out && lambda > 0, "bad argument");
    DN_REQUIRE(data_term == DN_DATA_L2 || data_term == DN_DATA_L1, "bad data_term");
    int rc = energy_current(v, lambda, false, data_term);
    if (rc) return rc;
    return read_energy(v, out);
}

int dn_regularize(dn_volume *v, const dn_reg_params *prm, const float *u0, const float *p0, dn_reg_stats *out)
{
    DN_REQUIRE(v, "null volume");
    int rc = validate(prm);
    if (rc) return rc;
    DN_REQUIRE(prm->init != DN_INIT_GIVEN || u0, "init GIVEN needs u0");
    DN_REQUIRE(prm->storage == DN_F32 || v->prm.state16, "16-bit storage needs a volume created with state16");
    hipStream_t st = v->stream;
    if ((rc = build_masks(v))) return rc;
    const int64_t n = v->nb * kBlockVox, ps = v->cap_blocks * kBlockVox;
    const int storage = prm->storage;
    // initial state
    if (prm->init == DN_INIT_ZERO) {
        if ((rc = zero_state(v))) return rc;
    } else if (prm->init == DN_INIT_GIVEN) {
        if (n > 0) {
            DN_HIP(hipMemcpyAsync(v->u, u0, n * 4, hipMemcpyDeviceToDevice, st));
            DN_HIP(hipMemcpyAsync(v->ubar[v->cur], u0, n * 4, hipMemcpyDeviceToDevice, st));
            for (int a = 0; a < 3; ++a) {
                if (p0) {
                    DN_HIP(hipMemcpyAsync(v->p[v->cur] + a * ps, p0 + a * n, n * 4, hipMemcpyDeviceToDevice, st));
                } else if ((rc = fill<float>(st, v->p[v->cur] + a * ps, n, 0.f))) {
                    return rc;
                }
            }
        }
        v->state_storage = DN_F32;
    } else if (prm->init == DN_INIT_CONTINUE) {
        // a 16-bit run ended with an FP32 sweep: continue from its output
        v->state_storage = DN_F32;
        const int64_t first = v->nb_state < v->nb ? v->nb_state : v->nb;
        const int64_t cnt = (v->nb - first) * kBlockVox;
        if (cnt > 0) {
            DN_HIP(hipMemcpyAsync(v->u + first * kBlockVox, v->f + first * kBlockVox, cnt * 4,
                                  hipMemcpyDeviceToDevice, st));
            DN_HIP(hipMemcpyAsync(v->ubar[v->cur] + first * kBlockVox, v->f + first * kBlockVox, cnt * 4,
                                  hipMemcpyDeviceToDevice, st));
            for (int a = 0; a < 3; ++a)
                if ((rc = fill<float>(st, v->p[v->cur] + a * ps + first * kBlockVox, cnt, 0.f))) return rc;
        }
    }
    if (prm->init != DN_INIT_KEEP || v->acc_tau <= 0.0) {
        v->acc_tau = prm->tau;
        v->acc_sigma = prm->sigma;
    }
    // the stochastic rounding restarts its seeds with the solve (a call that
    // keeps the state continues them), so equal calls give equal results
    if (prm->init != DN_INIT_KEEP) v->lowp_iter = 0;
    int kernel = prm->kernel;
    bool fresh16 = false;     // the 16-bit state was just demoted from FP32
    if (storage != DN_F32) {
        if (kernel != DN_K_FUSED256) kernel = DN_K_FUSED;
        if (v->state_storage != storage) {
            // the FP32 state (zero, given or an earlier FP32 run) is demoted
            if (v->state_storage != DN_F32) {
                set_error("cannot continue a %s state with another 16-bit storage",
                          v->state_storage == DN_F16 ? "FP16" : "BF16");
                return DN_E_INVALID;
            }
            rc = storage == DN_F16 ? demote_state<SF16>(v) : demote_state<SBF16>(v);
            if (rc) return rc;
            v->state_storage = storage;
            fresh16 = true;
        }
        if (prm->kernel == DN_K_AUTO && v->nb > 0) {
            if (fresh16) {
                rc = storage == DN_F16 ? autotune_lowp<SF16>(v, prm, storage, &kernel)
                                       : autotune_lowp<SBF16>(v, prm, storage, &kernel);
                if (rc) return rc;
            } else {
                AutoChoice found;
                if (find_choice(g_auto_lowp, tune_key(v, storage * 64 + size_bucket(v->nb)), &found)) {
                    kernel = found.kernel;
                    v->layout = found.layout;
                }
            }
        }
    } else {
        // a 16-bit run always ends with an FP32 sweep: continue from its output
        v->state_storage = DN_F32;
        if (kernel == DN_K_AUTO && v->nb > 0) {
            if (prm->init == DN_INIT_ZERO) {
                if ((rc = autotune_single(v, prm, &kernel))) return rc;
            } else {
                AutoChoice found;
                if (find_choice(g_auto_kernel, tune_key(v, size_bucket(v->nb)), &found)) {
                    kernel = found.kernel;
                    v->layout = found.layout;
                } else {
                    kernel = DN_K_FUSED;
                }
            }
        }
    }
    dn_reg_stats stats{};
    double ed[2] = {0, 0};
    int it = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    DN_HIP(hipEventCreate(&ev0));
    DN_HIP(hipEventCreate(&ev1));
    DN_HIP(hipEventRecord(ev0, st));
    dn_reg_params step_prm = *prm;
    bool last_refined = false;   // the last 16-bit iteration also wrote the FP32 state
    for (; it < prm->iters && v->nb > 0; ++it) {
        if (prm->gamma > 0.0) {
            // accelerated schedule: this iteration's (sigma_n, tau_n, theta_n)
            const double th = 1.0 / std::sqrt(1.0 + 2.0 * prm->gamma * v->acc_tau);
            step_prm.tau = v->acc_tau;
            step_prm.sigma = v->acc_sigma;
            step_prm.theta = th;
            v->acc_tau = th * v->acc_tau;
            v->acc_sigma = v->acc_sigma / th;
        }
        if (storage == DN_F32) {
            rc = step_f32(v, &step_prm, kernel);
        } else {
            bool refine = (prm->refine_every > 0 && (it + 1) % prm->refine_every == 0) || it + 1 == prm->iters;
            rc = storage == DN_F16 ? step_lowp<SF16>(v, &step_prm, refine, kernel)
                                   : step_lowp<SBF16>(v, &step_prm, refine, kernel);
            last_refined = refine;
        }
        if (rc) return rc;
        if (prm->gap_every > 0 && (it + 1) % prm->gap_every == 0 && it + 1 < prm->iters) {
            if ((rc = energy_current(v, prm->lambda, false, prm->data_term))) return rc;
            if ((rc = read_energy(v, ed))) return rc;
            double gap = ed[0] - ed[1];
            if (!std::isfinite(gap)) { set_error("non-finite gap at iteration %d", it + 1); return DN_E_NUMERIC; }
            if (prm->gap_tol > 0 && gap <= prm->gap_tol * ed[0]) { ++it; stats.converged = 1; break; }
        }
    }
    stats.iters_run = it;
    v->nb_state = v->nb;
    if (storage != DN_F32 && it > 0 && !last_refined) {
        // stopped early (gap_tol) between sweeps: the FP32 buffers take the
        // current 16-bit state
        rc = storage == DN_F16 ? promote_state<SF16>(v) : promote_state<SBF16>(v);
        if (rc) return rc;
    }
    DN_HIP(hipEventRecord(ev1, st));
    DN_HIP(hipEventSynchronize(ev1));
    {
        float ms = 0.f;
        DN_HIP(hipEventElapsedTime(&ms, ev0, ev1));
        stats.ms_loop = ms;
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
    // after a 16-bit run the FP32 buffers hold the result: the output of
    // the last sweep, or the promoted 16-bit state after an early stop
    if ((rc = energy_current(v, prm->lambda, true, prm->data_term))) return rc;
    if ((rc = read_energy(v, ed))) return rc;
    stats.energy = ed[0];
    stats.dual = ed[1];
    stats.gap = ed[0] - ed[1];
    stats.rel_gap = ed[0] != 0.0 ? stats.gap / ed[0] : 0.0;
    if (prm->gap_tol > 0 && stats.gap <= prm->gap_tol * ed[0]) stats.converged = 1;
    stats.kernel_used = kernel;
    stats.layout_used = v->layout;
    if (out) *out = stats;
    if (!std::isfinite(stats.gap)) { set_error("non-finite energy"); return DN_E_NUMERIC; }
    return DN_OK;
}

}  // extern "C"
