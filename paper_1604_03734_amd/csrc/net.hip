// Learned warm start: a 3-layer 3x3x3 convolutional network on 10^3 tiles
// (an 8^3 block plus a one-voxel halo), 2 -> 16 -> 16 -> 1 channels, ReLU,
// "same" zero padding inside the tile.
//
// Training path (forward, input gradient, weight gradient): one implicit
// GEMM launch per layer on v_mfma_f32_16x16x16_bf16 (bfloat16 operands,
// float32 accumulation; one MFMA = 16 voxels x 16 output channels x 16 input
// channels of one tap), activations stored channel-last in bfloat16,
// [tile][1000][16], unused channels zero.
//
// Inference path (warm start): one fused launch per axis, k_net_infer, on
// v_mfma_f32_16x16x32_bf16 with all activations in LDS and the weights in
// registers.  Its layer loops read one 1 KiB activation operand from LDS per
// MFMA; at the measured ~140 B/clk of 16-byte LDS reads per CU that bounds
// it near half the matrix peak.
#include <cstring>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "dn_internal.h"

namespace dn {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kT = 1000;      // voxels of a 10^3 tile
constexpr int kC = 16;        // channels of a stored activation
constexpr int kTaps = 27;
constexpr int kWPack = kTaps * kC * kC;   // one packed layer: [tap][co][ci]
constexpr int kMT = 63;       // 16-voxel row tiles covering 1000 voxels

__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float(uint32_t(v) << 16); }

// voxel v of a tile -> coordinates; neighbour through tap t (offset -1..1)
__device__ __forceinline__ int tap_neighbour(int v, int t)
{
    int x = v % 10, y = (v / 10) % 10, z = v / 100;
    x += t % 3 - 1; y += (t / 3) % 3 - 1; z += t / 9 - 1;
    if (x < 0 || x > 9 || y < 0 || y > 9 || z < 0 || z > 9) return -1;
    return (z * 10 + y) * 10 + x;
}

__device__ __forceinline__ void load_tile(uint16_t *dst, const uint16_t *src)
{
    const uint4 *s = reinterpret_cast<const uint4 *>(src);
    uint4 *d = reinterpret_cast<uint4 *>(dst);
    for (int i = threadIdx.x; i < kT * kC / 8; i += blockDim.x) d[i] = s[i];
}

// One convolution layer on one tile per workgroup (256 threads = 4 waves).
//   Y[v][co] = bias[co] + sum_t sum_ci W[t][co][ci] X[v + off(t)][ci]
// then optional ReLU, optional gate (multiply by [G[v][co] > 0], the ReLU
// derivative of the backward pass), stored as bfloat16 (Y) and/or channel 0
// as float (Yf).  With Wlo the weights are the pair Wp + Wlo (a second
// bfloat16 holding what the first rounded off).
__global__ __launch_bounds__(256) void k_conv(const uint16_t *__restrict__ X, int64_t n,
                                              const uint16_t *__restrict__ Wp, const uint16_t *__restrict__ Wlo,
                                              const float *__restrict__ bias, int relu,
                                              const uint16_t *__restrict__ gate, uint16_t *__restrict__ Y,
                                              float *__restrict__ Yf)
{
    __shared__ __align__(16) uint16_t sx[kT * kC];
    __shared__ __align__(16) uint16_t sw[kWPack];
    __shared__ __align__(16) uint16_t swl[kWPack];
    const int64_t tile = blockIdx.x;
    if (tile >= n) return;
    load_tile(sx, X + tile * kT * kC);
    {
        const uint4 *s = reinterpret_cast<const uint4 *>(Wp);
        uint4 *d = reinterpret_cast<uint4 *>(sw);
        for (int i = threadIdx.x; i < kWPack / 8; i += blockDim.x) d[i] = s[i];
        if (Wlo) {
            const uint4 *sl = reinterpret_cast<const uint4 *>(Wlo);
            uint4 *dl = reinterpret_cast<uint4 *>(swl);
            for (int i = threadIdx.x; i < kWPack / 8; i += blockDim.x) dl[i] = sl[i];
        }
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 15, kg = lane >> 4;
    const float bv = bias ? bias[i] : 0.0f;
    for (int mt = wave; mt < kMT; mt += 4) {
        const int v = mt * 16 + i;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        for (int t = 0; t < kTaps; ++t) {
            v4s a = {0, 0, 0, 0};
            if (v < kT) {
                int nvx = tap_neighbour(v, t);
                if (nvx >= 0) a = *reinterpret_cast<const v4s *>(&sx[nvx * kC + 4 * kg]);
            }
            v4s b = *reinterpret_cast<const v4s *>(&sw[(t * kC + i) * kC + 4 * kg]);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
            if (Wlo) {
                v4s bl = *reinterpret_cast<const v4s *>(&swl[(t * kC + i) * kC + 4 * kg]);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bl, acc, 0, 0, 0);
            }
        }
        for (int r = 0; r < 4; ++r) {
            const int vo = mt * 16 + 4 * kg + r;
            if (vo >= kT) continue;
            float y = acc[r] + bv;
            if (relu) y = y > 0.f ? y : 0.f;
            const int64_t o = (tile * kT + vo) * kC + i;
            if (gate) {
                uint16_t g = gate[o];
                if ((g & 0x8000u) || (g & 0x7FFFu) == 0) y = 0.f;
            }
            if (Y) Y[o] = f2bf(y);
            if (Yf && i == 0) Yf[tile * kT + vo] = y;
        }
    }
}

// Weight and bias gradient of one layer: dW[t][co][ci] = sum over tiles and
// voxels of X[v + off(t)][ci] dY[v][co]; db[co] = sum dY[v][co].  Each
// workgroup accumulates its tiles and writes one partial
// [27*256 + 16] floats; k_grad_reduce sums the partials in a fixed order.
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t *__restrict__ X, const uint16_t *__restrict__ dY,
                                               int64_t n, float *__restrict__ partials)
{
    __shared__ __align__(16) uint16_t sx[kT * kC];
    __shared__ __align__(16) uint16_t sd[kT * kC];
    __shared__ float sb[256];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 15, kg = lane >> 4;
    v4f acc[7];
    for (int j = 0; j < 7; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    for (int64_t tile = blockIdx.x; tile < n; tile += gridDim.x) {
        load_tile(sx, X + tile * kT * kC);
        load_tile(sd, dY + tile * kT * kC);
        __syncthreads();
        for (int ks = 0; ks < kMT; ++ks) {
            const int v0 = ks * 16 + 4 * kg;
            v4s b;
            for (int q = 0; q < 4; ++q) b[q] = (v0 + q < kT) ? short(sd[(v0 + q) * kC + i]) : short(0);
            for (int j = 0; j < 7; ++j) {
                const int t = wave + 4 * j;
                if (t >= kTaps) break;
                v4s a;
                for (int q = 0; q < 4; ++q) {
                    int nv = (v0 + q < kT) ? tap_neighbour(v0 + q, t) : -1;
                    a[q] = nv >= 0 ? short(sx[nv * kC + i]) : short(0);
                }
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
            }
        }
        // bias: channel c = tid % 16 summed over voxels tid/16, +16, ...
        for (int v = threadIdx.x >> 4; v < kT; v += 16) bsum += bf2f(sd[v * kC + (threadIdx.x & 15)]);
        __syncthreads();
    }
    float *out = partials + int64_t(blockIdx.x) * (kWPack + kC);
    // D layout: lane holds rows (ci) 4*kg + r, column (co) i
    for (int j = 0; j < 7; ++j) {
        const int t = wave + 4 * j;
        if (t >= kTaps) break;
        for (int r = 0; r < 4; ++r) out[(t * kC + i) * kC + 4 * kg + r] = acc[j][r];
    }
    sb[threadIdx.x] = bsum;
    __syncthreads();
    if (threadIdx.x < kC) {
        float s = 0.f;
        for (int k = 0; k < 16; ++k) s += sb[k * 16 + threadIdx.x];
        out[kWPack + threadIdx.x] = s;
    }
}

// First level of the partial reduction: chunk c of the partials (parts
// [c*per, (c+1)*per)) summed in order, per entry, into out[c][...].
__global__ void k_sum_parts(const float *__restrict__ partials, int nparts, int per, float *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (k >= kWPack + kC) return;
    float s = 0.f;
    const int p1 = min(nparts, (c + 1) * per);
    for (int p = c * per; p < p1; ++p) s += partials[int64_t(p) * (kWPack + kC) + k];
    out[int64_t(c) * (kWPack + kC) + k] = s;
}

// Sum the per-workgroup partials (fixed order) into the canonical parameter
// layout W[co][ci][tap], b[co] of a layer with cout x cin real channels.
__global__ void k_grad_reduce(const float *__restrict__ partials, int nparts, int cout, int cin,
                              float *__restrict__ gW, float *__restrict__ gb)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = cout * cin * kTaps;
    if (k < nw) {
        int co = k / (cin * kTaps), ci = (k / kTaps) % cin, t = k % kTaps;
        float s = 0.f;
        for (int p = 0; p < nparts; ++p) s += partials[int64_t(p) * (kWPack + kC) + (t * kC + co) * kC + ci];
        gW[k] = s;
    } else if (k < nw + cout) {
        int co = k - nw;
        float s = 0.f;
        for (int p = 0; p < nparts; ++p) s += partials[int64_t(p) * (kWPack + kC) + kWPack + co];
        gb[co] = s;
    }
}

// Pack the float parameters into bfloat16 [tap][co][ci] layers, zero padded
// to 16x16; flipped = 1 gives the input-gradient weights
// W'[t][a][b] = W[26 - t][b][a]; flipped = 2 gives the unflipped low part
// bfloat16(W - bfloat16(W)) (layer 1 runs on the pair hi + lo).
__global__ void k_pack(const float *__restrict__ W, int cout, int cin, int flipped, uint16_t *__restrict__ out)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kWPack) return;
    int t = k / (kC * kC), a = (k / kC) % kC, b = k % kC;
    float val = 0.f;
    if (flipped != 1) {
        if (a < cout && b < cin) val = W[(a * cin + b) * kTaps + t];
        if (flipped == 2) val -= bf2f(f2bf(val));
    } else {
        // a indexes the forward input channel, b the forward output channel
        if (b < cout && a < cin) val = W[(b * cin + a) * kTaps + (kTaps - 1 - t)];
    }
    out[k] = f2bf(val);
}

// float tiles [n][2][1000] -> bfloat16 [n][1000][16]
__global__ void k_tiles_to_bf16(const float *__restrict__ tiles, int64_t n, uint16_t *__restrict__ X)
{
    int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n * kT) return;
    int64_t tile = k / kT;
    int v = int(k % kT);
    uint16_t out[16];
    out[0] = f2bf(tiles[tile * 2 * kT + v]);
    out[1] = f2bf(tiles[tile * 2 * kT + kT + v]);
    for (int c = 2; c < 16; ++c) out[c] = 0;
    uint4 *d = reinterpret_cast<uint4 *>(X + k * kC);
    d[0] = *reinterpret_cast<uint4 *>(&out[0]);
    d[1] = *reinterpret_cast<uint4 *>(&out[8]);
}

__device__ __forceinline__ int64_t halo_vox(const int32_t *nb27, int hx, int hy, int hz)
{
    int dx = hx < 0 ? -1 : (hx > 7 ? 1 : 0);
    int dy = hy < 0 ? -1 : (hy > 7 ? 1 : 0);
    int dz = hz < 0 ? -1 : (hz > 7 ? 1 : 0);
    int32_t id = nb27[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
    if (id < 0) return -1;
    return int64_t(id) * kBlockVox + ((hx - 8 * dx) + 8 * (hy - 8 * dy) + 64 * (hz - 8 * dz));
}

// Input tiles of blocks [first, first + n) of the list (or of the pool if
// blocks == nullptr): channel 0 f, channel 1 log(1 + w) / log(101); 0 for
// voxels of unallocated neighbours.  Either float [n][2][1000] or
// bfloat16 channel-last [n][1000][16].
// perm exchanges the tile's x axis with the volume's y (1) or z (2) axis.
__global__ void k_gather(const int32_t *__restrict__ nbr, const float *__restrict__ f, const float *__restrict__ w,
                         const int32_t *__restrict__ blocks, int64_t first, int64_t n, float *__restrict__ tiles,
                         uint16_t *__restrict__ X, int perm)
{
    int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n * kT) return;
    int64_t i = k / kT;
    int v = int(k % kT);
    int64_t b = blocks ? blocks[first + i] : first + i;
    int x = v % 10, y = (v / 10) % 10, z = v / 100;
    if (perm == 1) { int s = x; x = y; y = s; }
    if (perm == 2) { int s = x; x = z; z = s; }
    int64_t j = halo_vox(nbr + b * kNbr, x - 1, y - 1, z - 1);
    float fv = 0.f, wv = 0.f;
    if (j >= 0) {
        fv = f[j];
        wv = float(log(1.0 + double(w[j])) / log(101.0));
    }
    if (tiles) {
        tiles[i * 2 * kT + v] = fv;
        tiles[i * 2 * kT + kT + v] = wv;
    }
    if (X) {
        uint16_t out[16];
        out[0] = f2bf(fv);
        out[1] = f2bf(wv);
        for (int c = 2; c < 16; ++c) out[c] = 0;
        uint4 *d = reinterpret_cast<uint4 *>(X + k * kC);
        d[0] = *reinterpret_cast<uint4 *>(&out[0]);
        d[1] = *reinterpret_cast<uint4 *>(&out[8]);
    }
}

__device__ __forceinline__ int centre_of(int v) { return ((v / 64 + 1) * 10 + ((v / 8) % 8 + 1)) * 10 + (v % 8 + 1); }

// Number of mask entries set: workgroup g sums its 4096-entry chunk in a
// fixed order (thread-strided, then a tree) into part[g]; then one
// workgroup sums the parts in order.
__global__ void k_mask_part(const float *__restrict__ mask, int64_t n, double *__restrict__ part)
{
    __shared__ double s[256];
    const int64_t base = int64_t(blockIdx.x) * 4096;
    double acc = 0.0;
    for (int k = threadIdx.x; k < 4096; k += 256)
        if (base + k < n) acc += mask[base + k];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void k_mask_count(const double *__restrict__ part, int64_t nparts, double *__restrict__ out)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < nparts; k += 256) acc += part[k];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

// Loss of one tile per workgroup (512 threads, one per centre voxel) and the
// output gradient dY3 (bfloat16, channel 0 only).
__global__ __launch_bounds__(512) void k_loss(const float *__restrict__ tiles, const float *__restrict__ R,
                                              const float *__restrict__ targets, const float *__restrict__ mask,
                                              const double *__restrict__ count, int64_t n, int kind,
                                              uint16_t *__restrict__ dY, double *__restrict__ tile_loss)
{
    __shared__ double sl[8];
    const int64_t tile = blockIdx.x;
    const int v = threadIdx.x;
    const double N = count[0] > 1.0 ? count[0] : 1.0;
    const int c = centre_of(v);
    const double m = mask[tile * 512 + v];
    double e = (kind == 0 ? double(tiles[tile * 2 * kT + c]) : 0.0) + double(R[tile * kT + c]) -
               double(targets[tile * 512 + v]);
    double l = m != 0.0 ? e * e / N : 0.0;
    // clear the tile's gradient, then write the centre voxels
    uint4 z = make_uint4(0, 0, 0, 0);
    uint4 *d = reinterpret_cast<uint4 *>(dY + tile * kT * kC);
    for (int k = threadIdx.x; k < kT * kC / 8; k += 512) d[k] = z;
    __syncthreads();
    if (m != 0.0) dY[(tile * kT + c) * kC] = f2bf(float(2.0 * e / N));
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
    if ((v & 63) == 0) sl[v >> 6] = l;
    __syncthreads();
    if (v == 0) {
        double s = 0.0;
        for (int k = 0; k < 8; ++k) s += sl[k];
        tile_loss[tile] = s;
    }
}

__global__ void k_sum_loss(const double *__restrict__ tl, int64_t n, double *__restrict__ out)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += 256) acc += tl[k];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    float gk = g[k];
    float mk = b1 * m[k] + (1.f - b1) * gk;
    float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// p0 = P(grad(u0) / delta) with the masked forward differences of Eq. (3)
__global__ __launch_bounds__(512) void k_warm_p(int64_t nb, int64_t ps, const int32_t *__restrict__ nbr,
                                                const uint8_t *__restrict__ emask, const float *__restrict__ u0,
                                                float inv_delta, float *__restrict__ p0)
{
    const int64_t b = blockIdx.x;
    const int t = threadIdx.x, lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
    const int64_t gi = b * kBlockVox + t;
    const int32_t *nb27 = nbr + b * kNbr;
    const uint8_t m = emask[gi];
    const float u = u0[gi];
    float g0 = (m & 2) ? u0[lx < 7 ? gi + 1 : halo_vox(nb27, 8, ly, lz)] - u : 0.f;
    float g1 = (m & 4) ? u0[ly < 7 ? gi + 8 : halo_vox(nb27, lx, 8, lz)] - u : 0.f;
    float g2 = (m & 8) ? u0[lz < 7 ? gi + 64 : halo_vox(nb27, lx, ly, 8)] - u : 0.f;
    g0 *= inv_delta; g1 *= inv_delta; g2 *= inv_delta;
    float nrm = sqrtf((g0 * g0 + g1 * g1) + g2 * g2);
    if (nrm > 1.f) { g0 /= nrm; g1 /= nrm; g2 /= nrm; }
    p0[gi] = g0; p0[gi + ps] = g1; p0[gi + 2 * ps] = g2;
}

// p0 onto the unit ball; u0 = f on Omega, 0 elsewhere
__global__ void k_warm_finish(int64_t n, int64_t ps, const uint8_t *__restrict__ emask, const float *__restrict__ f,
                              float *__restrict__ p0, float *__restrict__ u0)
{
    int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    float a = p0[g], b = p0[g + ps], c = p0[g + 2 * ps];
    float nrm = sqrtf((a * a + b * b) + c * c);
    if (nrm > 1.f) { a /= nrm; b /= nrm; c /= nrm; }
    p0[g] = a; p0[g + ps] = b; p0[g + 2 * ps] = c;
    u0[g] = (emask[g] & 1) ? f[g] : 0.f;
}

// The workspace of one network call (caller device memory): packed
// weights, activations of n tiles and, for training, their gradients and
// the weight-gradient partial sums.
struct NetWS {
    uint16_t *wpack, *x0, *h1, *h2, *d3, *d2, *d1;
    float *r, *parts, *chunks;
    double *misc, *tl, *mparts;
    int nparts, nchunks;
    int64_t nmask;
};
constexpr int kPartsPer = 16;   // partials summed per chunk
static NetWS carve_net(Bump &b, int64_t n, bool training)
{
    NetWS x{};
    const size_t act = size_t(n) * kT * kC;
    x.wpack = b.take<uint16_t>(size_t(6) * kWPack);
    x.x0 = b.take<uint16_t>(act);
    x.h1 = b.take<uint16_t>(act);
    x.h2 = b.take<uint16_t>(act);
    x.r = b.take<float>(size_t(n) * kT);
    if (training) {
        x.d3 = b.take<uint16_t>(act);
        x.d2 = b.take<uint16_t>(act);
        x.d1 = b.take<uint16_t>(act);
        x.nparts = int(n < 512 ? n : 512);
        x.nchunks = (x.nparts + kPartsPer - 1) / kPartsPer;
        x.parts = b.take<float>(size_t(x.nparts) * (kWPack + kC));
        x.chunks = b.take<float>(size_t(x.nchunks) * (kWPack + kC));
        x.misc = b.take<double>(8);
        x.tl = b.take<double>(size_t(n));
        x.nmask = (n * 512 + 4095) / 4096;
        x.mparts = b.take<double>(size_t(x.nmask));
    }
    return x;
}

static bool ws_ok(const void *ws) { return ws && (reinterpret_cast<uintptr_t>(ws) & 255) == 0; }

static inline unsigned grid1(int64_t n, int bs = 256) { return unsigned((n + bs - 1) / bs); }

// offsets of the layers in the canonical 8241-float parameter vector
constexpr int kW1 = 0, kB1 = 16 * 2 * 27, kW2 = kB1 + 16, kB2 = kW2 + 16 * 16 * 27, kW3 = kB2 + 16,
              kB3 = kW3 + 16 * 27;

// ---------------------------------------------------------------------------
// Fused inference: gather, three layers and the warm-start epilogue of one
// tile per iteration of a workgroup, activations in LDS only.  Every layer
// is an implicit GEMM on v_mfma_f32_16x16x32_bf16 (16 voxels x 16 output
// channels x 32 products of (tap, input channel)); the weights of all three
// layers stay in registers for the whole launch.

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

constexpr int kL1M = 2;       // layer 1: 27 taps x 2 channels = 54 of 64 K slots
constexpr int kL2M = 14;      // layer 2: 27 taps x 16 channels, two taps per MFMA
constexpr int kL3M = 2;       // layer 3: rows = the 9 (y, z) tap pairs, K = 3 x taps x 16 channels
// layer 1 runs on the weight pair hi + lo (bfloat16(W) and bfloat16(W -
// bfloat16(W))): its few input channels make the layer's output sensitive to
// the rounding of W1, and the second MFMA per K step costs little
constexpr int kLaneW = (2 * kL1M + kL2M + kL3M) * 64 * 8;

// Lane-ready weights [mfma][lane][8] (bfloat16).  The K slots of lane
// group g = lane / 16, entry j, of MFMA m: layer 1 -> tap 16m + 4g + j/2,
// channel j%2; layer 2 -> tap 2m + g/2, channel 8(g%2) + j; the output
// column (output channel) is lane % 16.  Layer 3 has one output channel, so
// its rows are taps instead: row n = 3 kz + ky (n < 9) is the (y, z) tap
// pair, and the K slots of MFMA m, group g are x tap kx = 2m + g/2 (kx < 3),
// channel 8(g%2) + j.  The activation operand uses the same map, so the
// products pair up whatever order the hardware sums them in.
__global__ void k_pack_lanes(const float *__restrict__ params, uint16_t *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kLaneW) return;
    const int j = k & 7, lane = (k >> 3) & 63, m = k >> 9;
    const int g = lane >> 4, n = lane & 15;
    float val = 0.f;
    if (m < kL1M || m >= kL1M + kL2M + kL3M) {
        const int ml = m < kL1M ? m : m - (kL1M + kL2M + kL3M);
        const int t = 16 * ml + 4 * g + (j >> 1), ci = j & 1;
        if (t < kTaps) val = params[kW1 + (n * 2 + ci) * kTaps + t];
        if (m >= kL1M) val -= bf2f(f2bf(val));
    } else if (m < kL1M + kL2M) {
        const int t = 2 * (m - kL1M) + (g >> 1), ci = 8 * (g & 1) + j;
        if (t < kTaps) val = params[kW2 + (n * 16 + ci) * kTaps + t];
    } else {
        const int kx = 2 * (m - kL1M - kL2M) + (g >> 1), ci = 8 * (g & 1) + j;
        if (kx < 3 && n < 9) val = params[kW3 + ci * kTaps + 3 * n + kx];
    }
    out[k] = f2bf(val);
}

// LDS activation: two planes of 8 channels, [2][1001][8] bfloat16 (row
// 1000 of each plane stays zero and stands for every neighbour outside the
// tile).  The 16 lanes of a 16-byte read take consecutive voxels of one
// plane, i.e. consecutive 16-byte chunks; the plane stride is 128 modulo
// 256 bytes, so the same voxels of the two planes fall in opposite halves
// of the banks.
constexpr int kPlane = 16256;              // bytes per plane, >= 1001 * 16
__device__ __forceinline__ int act_byte(int v, int half) { return half * kPlane + v * 16; }

__device__ __forceinline__ v8bf as_v8bf(v4u q) { return __builtin_bit_cast(v8bf, q); }

__host__ __device__ constexpr int tap_off(int t) { return (t % 3 - 1) + 10 * ((t / 3) % 3 - 1) + 100 * (t / 9 - 1); }

// Bit t (tap t = 9 kz + 3 ky + kx) set when the neighbour of tile voxel
// (x, y, z) through tap t lies inside the 10^3 tile.
__device__ __forceinline__ uint32_t tap_mask(int x, int y, int z)
{
    const uint32_t mx = (x > 0 ? 1u : 0u) | 2u | (x < 9 ? 4u : 0u);
    const uint32_t my = (y > 0 ? 1u : 0u) | 2u | (y < 9 ? 4u : 0u);
    const uint32_t mz = (z > 0 ? 1u : 0u) | 2u | (z < 9 ? 4u : 0u);
    const uint32_t X = mx * 0x01249249u;                       // kx pattern, 9 times
    const uint32_t ys = ((my & 1u) ? 0x7u : 0u) | ((my & 2u) ? 0x38u : 0u) | ((my & 4u) ? 0x1C0u : 0u);
    const uint32_t Y = ys * 0x00040201u;                       // 3 times, 9 bits apart
    const uint32_t Z = ((mz & 1u) ? 0x1FFu : 0u) | ((mz & 2u) ? 0x3FE00u : 0u) | ((mz & 4u) ? 0x7FC0000u : 0u);
    return X & Y & Z;
}

__device__ __forceinline__ v4u lds_row(const uint16_t *h, int byte)
{
    return *reinterpret_cast<const v4u *>(reinterpret_cast<const char *>(h) + byte);
}

// A K chain of NM MFMAs whose operands are loaded G at a time, one group
// ahead of the products that use them, so LDS latency overlaps the matrix
// work.  a_of(m) returns the activation operand of step m, b_of(m) the
// weight operand (a register, or an LDS read when kLdsB).
template <int NM, int G, bool kLdsB, class FA, class FB>
__device__ __forceinline__ v4f mfma_chain(FA a_of, FB b_of)
{
    constexpr int NG = (NM + G - 1) / G;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    v8bf qa[2][G], qb[2][G];
#pragma unroll
    for (int k = 0; k < G; ++k)
        if (k < NM) {
            qa[0][k] = a_of(k);
            if constexpr (kLdsB) qb[0][k] = b_of(k);
        }
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
        __builtin_amdgcn_sched_barrier(0);
        const int cur = gi & 1;
        if (gi + 1 < NG) {
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int m = (gi + 1) * G + k;
                if (m < NM) {
                    qa[cur ^ 1][k] = a_of(m);
                    if constexpr (kLdsB) qb[cur ^ 1][k] = b_of(m);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const int m = gi * G + k;
            if (m < NM) {
                v8bf bb;
                if constexpr (kLdsB) bb = qb[cur][k];
                else bb = b_of(m);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bb, qa[cur][k], acc, 0, 0, 0);
            }
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    return acc;
}

// Products are taken as W x A^T, so a lane holds 4 output channels
// (4g .. 4g+3) of voxel i of the row tile: bias + ReLU, then one 8-byte
// store per lane.
// (bias + ReLU rounded to bfloat16 by the hardware's round-to-nearest-even
// pair conversion, the same rounding as f2bf for these finite values)
typedef float v2f_t __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_act(uint16_t *h, int vo, int g, v4f acc, const float *bias4)
{
    if (vo < kT) {
        float y[4];
        for (int r = 0; r < 4; ++r) {
            const float a = acc[r] + bias4[r];
            y[r] = a > 0.f ? a : 0.f;
        }
        const uint2 pk = make_uint2(__builtin_bit_cast(uint32_t, __builtin_convertvector(v2f_t{y[0], y[1]}, v2bf_t)),
                                    __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f_t{y[2], y[3]}, v2bf_t)));
        *reinterpret_cast<uint2 *>(reinterpret_cast<char *>(h) + act_byte(vo, g >> 1) + 8 * (g & 1)) = pk;
    }
}

// Layer-1 input word of every voxel of the pool: the bfloat16 pair
// (f, log(1 + w) / log(101)), computed once for the three axes; the
// inference kernel reads its tiles from it through the neighbour table.
__global__ void k_voxel_pairs(const float *__restrict__ f, const float *__restrict__ w, int64_t n,
                              uint32_t *__restrict__ pair)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float wv = float(log(1.0 + double(w[i])) / log(101.0));
    pair[i] = uint32_t(f2bf(f[i])) | (uint32_t(f2bf(wv)) << 16);
}

// mode DN_WARM_DUAL: out = p0, component perm written on the centre (kept
// where m_perm = 1); mode DN_WARM_PRIMAL (perm 0): out = u0 =
// clamp(f + r, -1, 1) on Omega, 0 elsewhere.  Workgroups loop over tiles;
// the layer-1 input of the next tile is loaded while the current one is
// computed.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_net_infer(
    const int32_t *__restrict__ nbr, const uint32_t *__restrict__ pair, const float *__restrict__ f,
    const uint8_t *__restrict__ emask, int64_t nb, int perm, int mode, const uint16_t *__restrict__ lw,
    const float *__restrict__ params, int64_t ps, float *__restrict__ out)
{
    __shared__ __align__(16) uint16_t h1[2 * kPlane / 2];
    __shared__ __align__(16) uint16_t h2[2 * kPlane / 2];
    __shared__ __align__(16) uint32_t x0[kT + 4];
    __shared__ uint32_t okt[kMT * 16];   // tap masks of the tile voxels (0 past the tile)
    __shared__ uint16_t vt[kMT * 16];    // voxel of each (row tile, lane column)
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // Row tiles 0..31 hold the 512 voxels with x, y, z in 1..8, whose taps
    // all stay in the tile: x = 1..8 of rows y and y + 4 of one z plane
    // (640 bytes apart, so the 16 lanes' 16-byte reads cover the 64 LDS
    // banks once); tiles 32..62 hold the other 488 voxels in linear order
    // and 8 empty columns (kT).
    for (int v = tid; v < kMT * 16; v += 256) {
        okt[v] = v < kT ? tap_mask(v % 10, (v / 10) % 10, v / 100) : 0u;
        if (v >= kT) {
            vt[v] = uint16_t(kT);
            continue;
        }
        const int x = v % 10, y = (v / 10) % 10, z = v / 100;
        const bool iz = z >= 1 && z <= 8, iy = y >= 1 && y <= 8, ix = x >= 1 && x <= 8;
        int before = 64 * min(max(z - 1, 0), 8);                  // interior voxels before v
        if (iz) before += 8 * min(max(y - 1, 0), 8);
        if (iz && iy) before += min(max(x - 1, 0), 8);
        const int inner = 64 * (z - 1) + 16 * ((y - 1) % 4) + 8 * ((y - 1) / 4) + (x - 1);
        vt[(iz && iy && ix) ? inner : 512 + (v - before)] = uint16_t(v);
    }
    const int i = lane & 15, g = lane >> 4;
    const int half = g & 1, par = g >> 1;      // channel half and tap parity of this lane's K slots
    const v4u *lw4 = reinterpret_cast<const v4u *>(lw);
    v8bf W1[kL1M], W1l[kL1M], W2[kL2M], W3[kL3M];
    for (int m = 0; m < kL1M; ++m) W1[m] = as_v8bf(lw4[m * 64 + lane]);
    for (int m = 0; m < kL1M; ++m) W1l[m] = as_v8bf(lw4[(kL1M + kL2M + kL3M + m) * 64 + lane]);
    for (int m = 0; m < kL2M; ++m) W2[m] = as_v8bf(lw4[(kL1M + m) * 64 + lane]);
    for (int m = 0; m < kL3M; ++m) W3[m] = as_v8bf(lw4[(kL1M + kL2M + m) * 64 + lane]);
    float bias1[4], bias2[4];
    for (int r = 0; r < 4; ++r) {
        bias1[r] = params[kB1 + 4 * g + r];
        bias2[r] = params[kB2 + 4 * g + r];
    }
    const float bias3 = params[kB3];
    __builtin_amdgcn_s_waitcnt(0);
    if (tid < 8) reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(h1) + (tid >> 2) * kPlane + kT * 16)[tid & 3] = 0u;
    if (tid == 0) x0[kT] = 0u;

    // the layer-1 input of a tile, read from the pool's pair words through
    // the neighbour table (tile voxels of unallocated blocks give 0), the
    // next tile's while this one is computed
    constexpr int kGet = (kT + 255) / 256;
    uint32_t nxt[kGet];
    auto fetch = [&](int64_t bb) {
        const int32_t *nb27 = nbr + bb * kNbr;
        for (int e = 0; e < kGet; ++e) {
            const int k = tid + 256 * e;
            nxt[e] = 0u;
            if (k < kT) {
                int x = k % 10, y = (k / 10) % 10, z = k / 100;
                if (perm == 1) { const int sw = x; x = y; y = sw; }
                if (perm == 2) { const int sw = x; x = z; z = sw; }
                const int64_t j = halo_vox(nb27, x - 1, y - 1, z - 1);
                if (j >= 0) nxt[e] = pair[j];
            }
        }
    };
    if (blockIdx.x < nb) fetch(blockIdx.x);

    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        for (int e = 0; e < kGet; ++e)
            if (tid + 256 * e < kT) x0[tid + 256 * e] = nxt[e];
        __syncthreads();
        const int64_t bn = b + gridDim.x;
        if (bn < nb) fetch(bn);

        // layer 1: 2 -> 16, ReLU
        for (int mt = wave; mt < kMT; mt += 4) {
            const int v = vt[mt * 16 + i];
            const uint32_t ok = mt < 32 ? 0x7FFFFFFu : okt[v];
            v4u q[kL1M];
            for (int m = 0; m < kL1M; ++m)
                for (int e = 0; e < 4; ++e) {
                    const int t = 16 * m + 4 * g + e;
                    const int o = (t % 3 - 1) + 10 * ((t / 3) % 3 - 1) + 100 * (t / 9 - 1);
                    q[m][e] = x0[t < kTaps && ((ok >> t) & 1u) ? v + o : kT];
                }
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            for (int m = 0; m < kL1M; ++m) {
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W1[m], as_v8bf(q[m]), acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W1l[m], as_v8bf(q[m]), acc, 0, 0, 0);
            }
            store_act(h1, v, g, acc, bias1);
        }
        __syncthreads();

        // layer 2: 16 -> 16, ReLU; interior tiles read every tap at a fixed
        // offset from the voxel (the past-the-end tap 27 reads the zero row)
        for (int mt = wave; mt < kMT; mt += 4) {
            const int v = vt[mt * 16 + i];
            v4f acc;
            if (mt < 32) {
                const int base = act_byte(v, half), zero = act_byte(kT, half);
                acc = mfma_chain<kL2M, 5, false>(
                    [&](int m) {
                        const int addr = par ? (2 * m + 1 < kTaps ? base + 16 * tap_off(2 * m + 1) : zero)
                                             : base + 16 * tap_off(2 * m);
                        return as_v8bf(lds_row(h1, addr));
                    },
                    [&](int m) { return W2[m]; });
            } else {
                const uint32_t ok = okt[v];
                acc = mfma_chain<kL2M, 5, false>(
                    [&](int m) {
                        const int o = par ? tap_off(2 * m + 1) : tap_off(2 * m);
                        const int nv = ((ok >> (2 * m + par)) & 1u) ? v + o : kT;
                        return as_v8bf(lds_row(h1, act_byte(nv, half)));
                    },
                    [&](int m) { return W2[m]; });
            }
            store_act(h2, v, g, acc, bias2);
        }
        __syncthreads();

        // layer 3: 16 -> 1 on the centre 8^3, as partial sums over the x taps.
        // P[n][u] = sum over kx, ci of W3[ci][3n + kx] h2[u + kx - 1][ci] for
        // the 9 (y, z) tap pairs n and the 800 voxels u with x in 1..8 (rows
        // r = 10 z + y, 8 voxels each), one 16-voxel tile (two rows) per pair
        // of MFMAs; P goes to h1, which layer 2 has finished reading.
        float *P = reinterpret_cast<float *>(h1);
        for (int mt = wave; mt < 50; mt += 4) {
            const int r = 2 * mt + (i >> 3), u = 10 * r + (i & 7) + 1;
            const v4u z4 = {0u, 0u, 0u, 0u};
            const v4u q0 = lds_row(h2, act_byte(u - 1 + par, half));       // kx = par
            const v4u q1 = par ? z4 : lds_row(h2, act_byte(u + 1, half));  // kx = 2
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W3[0], as_v8bf(q0), acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W3[1], as_v8bf(q1), acc, 0, 0, 0);
            // lane: rows (tap pairs) 4g .. 4g+3 of column i
            for (int e = 0; e < 4; ++e)
                if (4 * g + e < 9) P[(4 * g + e) * 800 + 8 * r + (i & 7)] = acc[e];
        }
        __syncthreads();

        // the 9 pair sums of each centre voxel, then the epilogue
        for (int c = tid; c < kBlockVox; c += 256) {
            const int cx = c & 7, cy = (c >> 3) & 7, cz = c >> 6;
            float acc = 0.f;
            for (int n = 0; n < 9; ++n) {
                const int row = (cz + n / 3) * 10 + (cy + n % 3);   // (z + kz - 1 + 1, y + ky - 1 + 1)
                acc += P[n * 800 + 8 * row + cx];
            }
            int x = cx, y = cy, z = cz;
            if (perm == 1) { const int sw = x; x = y; y = sw; }
            if (perm == 2) { const int sw = x; x = z; z = sw; }
            const int64_t gi = b * kBlockVox + x + 8 * y + 64 * z;
            const float rv = acc + bias3;
            const uint8_t em = emask[gi];
            if (mode == DN_WARM_DUAL) {
                out[perm * ps + gi] = ((em >> (perm + 1)) & 1) ? rv : 0.f;
            } else {
                float uu = 0.f;
                if (em & 1) {
                    uu = f[gi] + rv;
                    uu = uu < -1.f ? -1.f : (uu > 1.f ? 1.f : uu);
                }
                out[gi] = uu;
            }
        }
        // P overwrote the zero row of h1's first plane
        if (tid < 4) reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(h1) + kT * 16)[tid] = 0u;
        __syncthreads();
    }
}

static int pack_all(hipStream_t st, const float *params, bool with_flipped, uint16_t *wp)
{
    hipLaunchKernelGGL(k_pack, dim3(grid1(kWPack)), dim3(256), 0, st, params + kW1, 16, 2, 0, wp);
    hipLaunchKernelGGL(k_pack, dim3(grid1(kWPack)), dim3(256), 0, st, params + kW2, 16, 16, 0, wp + kWPack);
    hipLaunchKernelGGL(k_pack, dim3(grid1(kWPack)), dim3(256), 0, st, params + kW3, 1, 16, 0, wp + 2 * kWPack);
    hipLaunchKernelGGL(k_pack, dim3(grid1(kWPack)), dim3(256), 0, st, params + kW1, 16, 2, 2, wp + 5 * kWPack);
    if (with_flipped) {
        hipLaunchKernelGGL(k_pack, dim3(grid1(kWPack)), dim3(256), 0, st, params + kW2, 16, 16, 1, wp + 3 * kWPack);
        hipLaunchKernelGGL(k_pack, dim3(grid1(kWPack)), dim3(256), 0, st, params + kW3, 1, 16, 1, wp + 4 * kWPack);
    }
    DN_HIP(hipGetLastError());
    return DN_OK;
}

// Forward of n tiles already in ws.x0 (packed weights in ws.wpack): h1, h2
// (bfloat16) and the residual r (float) of every tile voxel.
static int forward_tiles(hipStream_t st, const float *params, int64_t n, const NetWS &ws)
{
    if (n <= 0) return DN_OK;
    const uint16_t *wp = ws.wpack;
    uint16_t *x0 = ws.x0, *h1 = ws.h1, *h2 = ws.h2;
    hipLaunchKernelGGL(k_conv, dim3(unsigned(n)), dim3(256), 0, st, x0, n, wp, wp + 5 * kWPack, params + kB1, 1,
                       (const uint16_t *)nullptr, h1, (float *)nullptr);
    hipLaunchKernelGGL(k_conv, dim3(unsigned(n)), dim3(256), 0, st, h1, n, wp + kWPack, (const uint16_t *)nullptr,
                       params + kB2, 1, (const uint16_t *)nullptr, h2, (float *)nullptr);
    hipLaunchKernelGGL(k_conv, dim3(unsigned(n)), dim3(256), 0, st, h2, n, wp + 2 * kWPack, (const uint16_t *)nullptr,
                       params + kB3, 0, (const uint16_t *)nullptr, (uint16_t *)nullptr, ws.r);
    DN_HIP(hipGetLastError());
    return DN_OK;
}

// One forward pass of n tiles in the given workspace (sized by the caller).
static int forward_into(const float *tiles, int64_t n, const float *params, float *out, void *workspace,
                        size_t workspace_bytes, hipStream_t st)
{
    Bump bump(workspace, workspace_bytes);
    const NetWS ws = carve_net(bump, n, false);
    if (!bump.fits()) { set_error("network workspace too small"); return DN_E_CAPACITY; }
    int rc;
    if ((rc = pack_all(st, params, false, ws.wpack))) return rc;
    hipLaunchKernelGGL(k_tiles_to_bf16, dim3(grid1(n * kT)), dim3(256), 0, st, tiles, n, ws.x0);
    DN_HIP(hipGetLastError());
    if ((rc = forward_tiles(st, params, n, ws))) return rc;
    DN_HIP(hipMemcpyAsync(out, ws.r, size_t(n) * kT * 4, hipMemcpyDeviceToDevice, st));
    return DN_OK;
}

// Scratch of dn_net_forward_static: a file-scope device array, one copy per
// GPU, held until the process ends.  In host code its name is only a
// stand-in; the address each device's copy has is looked up once per device
// (with that device current) and kept.
constexpr size_t kNetStaticBytes = size_t(DN_NET_STATIC_TILES) * (size_t(kT) * kC * 2 * 3 + size_t(kT) * 4 + 1024) +
                                   size_t(6) * kWPack * 2 + 4096;
static __device__ __align__(256) unsigned char scratch[kNetStaticBytes];
constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mutex;

static int static_scratch(void **out)
{
    int dev = 0;
    DN_HIP(hipGetDevice(&dev));
    DN_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        DN_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        DN_REQUIRE(p && (reinterpret_cast<uintptr_t>(p) & 255) == 0, "static scratch misaligned");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DN_OK;
}

}  // namespace dn

using namespace dn;

extern "C" {

int dn_net_gather(dn_volume *v, const int32_t *blocks, int64_t n, int32_t perm, float *tiles)
{
    DN_REQUIRE(v && blocks && tiles && n >= 0 && perm >= 0 && perm <= 2, "bad argument");
    if (n == 0) return DN_OK;
    hipLaunchKernelGGL(k_gather, dim3(grid1(n * kT)), dim3(256), 0, v->stream, v->nbr, v->f, v->w, blocks,
                       int64_t(0), n, tiles, (uint16_t *)nullptr, int(perm));
    DN_HIP(hipGetLastError());
    return DN_OK;
}

size_t dn_net_bytes(int64_t n_tiles, int32_t training)
{
    if (n_tiles < 0 || (training != 0 && training != 1)) return 0;
    Bump b(nullptr, 0);
    carve_net(b, n_tiles, training != 0);
    return (b.off + 255) & ~size_t(255);
}

int dn_net_forward(const float *tiles, int64_t n, const float *params, float *out, void *workspace,
                   size_t workspace_bytes, void *stream)
{
    DN_REQUIRE(tiles && params && out && n >= 0, "bad argument");
    if (n == 0) return DN_OK;
    DN_REQUIRE(ws_ok(workspace), "the workspace must be non-null and 256-byte aligned");
    if (workspace_bytes < dn_net_bytes(n, 0)) {
        set_error("workspace of %zu bytes is short: %zu needed (dn_net_bytes)", workspace_bytes, dn_net_bytes(n, 0));
        return DN_E_CAPACITY;
    }
    return forward_into(tiles, n, params, out, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

int dn_net_forward_static(const float *tiles, int64_t n, const float *params, float *out, void *stream)
{
    DN_REQUIRE(tiles && params && out && n >= 0, "bad argument");
    if (n > DN_NET_STATIC_TILES) {
        set_error("dn_net_forward_static takes at most %d tiles per call (%lld given)", DN_NET_STATIC_TILES,
                  (long long)n);
        return DN_E_CAPACITY;
    }
    if (n == 0) return DN_OK;
    void *ws = nullptr;
    int rc = static_scratch(&ws);
    if (rc) return rc;
    return forward_into(tiles, n, params, out, ws, kNetStaticBytes, static_cast<hipStream_t>(stream));
}

int dn_net_loss_grad(const float *tiles, int64_t n, const float *params, const float *targets, const float *mask,
                     int32_t kind, float *grad, void *workspace, size_t workspace_bytes, double *loss_host,
                     void *stream)
{
    DN_REQUIRE(tiles && params && targets && mask && grad && n > 0 && (kind == 0 || kind == 1), "bad argument");
    DN_REQUIRE(ws_ok(workspace), "the workspace must be non-null and 256-byte aligned");
    if (workspace_bytes < dn_net_bytes(n, 1)) {
        set_error("workspace of %zu bytes is short: %zu needed (dn_net_bytes)", workspace_bytes, dn_net_bytes(n, 1));
        return DN_E_CAPACITY;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    Bump bump(workspace, workspace_bytes);
    const NetWS ws = carve_net(bump, n, true);
    int rc;
    if ((rc = pack_all(st, params, true, ws.wpack))) return rc;
    const int nparts = ws.nparts, per = kPartsPer, nchunks = ws.nchunks;
    float *chunks = ws.chunks;
    const dim3 cgrid(grid1(kWPack + kC), unsigned(nchunks));
    uint16_t *x0 = ws.x0, *h1 = ws.h1, *h2 = ws.h2;
    uint16_t *d3 = ws.d3, *d2 = ws.d2, *d1 = ws.d1;
    const uint16_t *wp = ws.wpack;
    double *cnt = ws.misc, *lsum = cnt + 1;
    float *parts = ws.parts;
    hipLaunchKernelGGL(k_tiles_to_bf16, dim3(grid1(n * kT)), dim3(256), 0, st, tiles, n, x0);
    DN_HIP(hipGetLastError());
    if ((rc = forward_tiles(st, params, n, ws))) return rc;
    const int64_t nmask = ws.nmask;
    hipLaunchKernelGGL(k_mask_part, dim3(unsigned(nmask)), dim3(256), 0, st, mask, n * 512, ws.mparts);
    hipLaunchKernelGGL(k_mask_count, dim3(1), dim3(256), 0, st, ws.mparts, nmask, cnt);
    hipLaunchKernelGGL(k_loss, dim3(unsigned(n)), dim3(512), 0, st, tiles, ws.r, targets, mask, cnt, n,
                       int(kind), d3, ws.tl);
    hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(256), 0, st, ws.tl, n, lsum);
    DN_HIP(hipGetLastError());
    // layer 3: weights from (h2, d3); input gradient d2 = conv(d3, W3 flipped) * [h2 > 0]
    hipLaunchKernelGGL(k_wgrad, dim3(nparts), dim3(256), 0, st, h2, d3, n, parts);
    hipLaunchKernelGGL(k_sum_parts, cgrid, dim3(256), 0, st, parts, nparts, per, chunks);
    hipLaunchKernelGGL(k_grad_reduce, dim3(grid1(16 * 27 + 1)), dim3(256), 0, st, chunks, nchunks, 1, 16,
                       grad + kW3, grad + kB3);
    hipLaunchKernelGGL(k_conv, dim3(unsigned(n)), dim3(256), 0, st, d3, n, wp + 4 * kWPack, (const uint16_t *)nullptr,
                       (const float *)nullptr, 0, h2, d2, (float *)nullptr);
    // layer 2
    hipLaunchKernelGGL(k_wgrad, dim3(nparts), dim3(256), 0, st, h1, d2, n, parts);
    hipLaunchKernelGGL(k_sum_parts, cgrid, dim3(256), 0, st, parts, nparts, per, chunks);
    hipLaunchKernelGGL(k_grad_reduce, dim3(grid1(16 * 16 * 27 + 16)), dim3(256), 0, st, chunks, nchunks, 16, 16,
                       grad + kW2, grad + kB2);
    hipLaunchKernelGGL(k_conv, dim3(unsigned(n)), dim3(256), 0, st, d2, n, wp + 3 * kWPack, (const uint16_t *)nullptr,
                       (const float *)nullptr, 0, h1, d1, (float *)nullptr);
    // layer 1
    hipLaunchKernelGGL(k_wgrad, dim3(nparts), dim3(256), 0, st, x0, d1, n, parts);
    hipLaunchKernelGGL(k_sum_parts, cgrid, dim3(256), 0, st, parts, nparts, per, chunks);
    hipLaunchKernelGGL(k_grad_reduce, dim3(grid1(16 * 2 * 27 + 16)), dim3(256), 0, st, chunks, nchunks, 16, 2,
                       grad + kW1, grad + kB1);
    DN_HIP(hipGetLastError());
    if (loss_host) {
        double h = 0.0;
        DN_HIP(hipMemcpyAsync(&h, lsum, 8, hipMemcpyDeviceToHost, st));
        DN_HIP(hipStreamSynchronize(st));
        *loss_host = h;
    }
    return DN_OK;
}

int dn_net_adam(float *params, const float *grad, float *m, float *v, int64_t n, float lr, float beta1, float beta2,
                float eps, int32_t step, void *stream)
{
    DN_REQUIRE(params && grad && m && v && n > 0 && step >= 1, "bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    float c1 = 1.f - std::pow(beta1, float(step)), c2 = 1.f - std::pow(beta2, float(step));
    hipLaunchKernelGGL(k_adam, dim3(grid1(n)), dim3(256), 0, st, params, grad, m, v, n, lr, beta1, beta2, eps, c1, c2);
    DN_HIP(hipGetLastError());
    return DN_OK;
}

size_t dn_warm_start_bytes(int64_t n_blocks)
{
    if (n_blocks < 0) return 0;
    Bump b(nullptr, 0);
    b.take<uint16_t>(size_t(kLaneW));
    b.take<uint32_t>(size_t(n_blocks) * kBlockVox);
    return (b.off + 255) & ~size_t(255);
}

int dn_net_warm_start(dn_volume *v, const float *params, int32_t mode, double delta, float *u0, float *p0,
                      void *workspace, size_t workspace_bytes)
{
    DN_REQUIRE(v && params && u0 && (mode == DN_WARM_PRIMAL || mode == DN_WARM_DUAL), "bad argument");
    DN_REQUIRE(mode == DN_WARM_DUAL ? p0 != nullptr : delta > 0, "dual mode needs p0; primal mode needs delta > 0");
    hipStream_t st = v->stream;
    int rc;
    if ((rc = build_masks(v))) return rc;
    if (v->nb == 0) return DN_OK;
    DN_REQUIRE(ws_ok(workspace), "the workspace must be non-null and 256-byte aligned");
    if (workspace_bytes < dn_warm_start_bytes(v->nb)) {
        set_error("workspace of %zu bytes is short: %zu needed (dn_warm_start_bytes)", workspace_bytes,
                  dn_warm_start_bytes(v->nb));
        return DN_E_CAPACITY;
    }
    Bump bump(workspace, workspace_bytes);
    uint16_t *lanew = bump.take<uint16_t>(size_t(kLaneW));
    uint32_t *vp = bump.take<uint32_t>(size_t(v->nb) * kBlockVox);
    hipLaunchKernelGGL(k_pack_lanes, dim3(grid1(kLaneW)), dim3(256), 0, st, params, lanew);
    DN_HIP(hipGetLastError());
    int cus = 0;
    DN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, v->device));
    // two workgroups fit a compute unit (64 KiB of LDS each); each loops over tiles
    const unsigned grid = unsigned(std::min<int64_t>(v->nb, int64_t(2) * (cus > 0 ? cus : 1)));
    const int64_t ps = v->nb * int64_t(kBlockVox);
    const int axes = mode == DN_WARM_DUAL ? 3 : 1;
    hipLaunchKernelGGL(k_voxel_pairs, dim3(grid1(ps)), dim3(256), 0, st, v->f, v->w, ps, vp);
    for (int a = 0; a < axes; ++a) {
        hipLaunchKernelGGL(k_net_infer, dim3(grid), dim3(256), 0, st, v->nbr, vp, v->f, v->emask, v->nb,
                           mode == DN_WARM_DUAL ? a : 0, int(mode), lanew, params, ps,
                           mode == DN_WARM_DUAL ? p0 : u0);
        DN_HIP(hipGetLastError());
    }
    if (mode == DN_WARM_DUAL) {
        hipLaunchKernelGGL(k_warm_finish, dim3(grid1(ps)), dim3(256), 0, st, ps, ps, v->emask, v->f, p0, u0);
        DN_HIP(hipGetLastError());
    } else if (p0) {
        hipLaunchKernelGGL(k_warm_p, dim3(unsigned(v->nb)), dim3(512), 0, st, v->nb, ps, v->nbr, v->emask, u0,
                           float(1.0 / delta), p0);
        DN_HIP(hipGetLastError());
    }
    return DN_OK;
}

}  // extern "C"
