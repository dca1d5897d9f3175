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
// Inference path (warm start): one fused launch per axis, k_net_fwd, on
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
// Training layouts: an activation channel-first on the tile's 10^3 grid
// padded by one zero voxel on every side (12^3 = 1728 entries per channel,
// index (x+1) + 12 (y+1) + 144 (z+1)); a gradient channel-first on the
// compact rows of that grid (the 100 rows (y, z) of 12 entries, padding
// entries x = -1 and x = 10 zero, index (x+1) + 12 (10 z + y), 1216 entries
// with the tail zero).
constexpr int kPadVox = 1728;
// offsets of the layers in the canonical 8241-float parameter vector
constexpr int kW1 = 0, kB1 = 16 * 2 * 27, kW2 = kB1 + 16, kB2 = kW2 + 16 * 16 * 27, kW3 = kB2 + 16,
              kB3 = kW3 + 16 * 27;
constexpr int kRowVox = 1216;

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

// Pack the float parameters into bfloat16 [tap][co][ci] layers, zero padded
// to 16x16; lo = 1 gives the low part bfloat16(W - bfloat16(W)) (layer 1
// runs on the pair hi + lo).
__global__ void k_pack(const float *__restrict__ W, int cout, int cin, int lo, uint16_t *__restrict__ out)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kWPack) return;
    int t = k / (kC * kC), a = (k / kC) % kC, b = k % kC;
    float val = 0.f;
    if (a < cout && b < cin) val = W[(a * cin + b) * kTaps + t];
    if (lo) val -= bf2f(f2bf(val));
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


// Number of mask entries set: workgroup g sums its 4096-entry chunk in a
// fixed order (thread-strided, then a tree) into part[g]; then one
// workgroup sums the parts in order.
// The gradient of all 8241 parameters from the per-workgroup partials of
// the three layers (parts[layer][p][27 * 256 + 16]), written to the
// canonical parameter layout and scaled by 1 / N (the partials are of the
// loss before its division by N: every entry is linear in d3).  The sum over p has a fixed order: a
// workgroup takes 32 consecutive partial entries (contiguous reads across
// its threads), its 8 thread groups add consecutive eighths of the
// partials (each in order, eight loads in flight), then the eight group
// sums are added in group order.
constexpr int kFinalEntries = 32, kFinalGroups = 8;
__global__ __launch_bounds__(256) void k_grad_final(const float *__restrict__ parts, int nparts,
                                                    const double *__restrict__ tile_loss,
                                                    const double *__restrict__ tile_count, int64_t ntiles,
                                                    double *__restrict__ loss, float *__restrict__ grad)
{
    __shared__ float sg[kFinalGroups][kFinalEntries];
    __shared__ double sl[256], sc[256];
    // N = max(1, sum of the mask) and the loss, the same fixed-order sums
    // in every workgroup; workgroup 0 writes loss[0] = squared errors / N,
    // loss[1] = 1 / N
    {
        double l = 0.0, c = 0.0;
        for (int64_t k = threadIdx.x; k < ntiles; k += 256) {
            l += tile_loss[k];
            c += tile_count[k];
        }
        sl[threadIdx.x] = l;
        sc[threadIdx.x] = c;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                sl[threadIdx.x] += sl[threadIdx.x + h];
                sc[threadIdx.x] += sc[threadIdx.x + h];
            }
            __syncthreads();
        }
    }
    const double N = sc[0] > 1.0 ? sc[0] : 1.0, inv_n = 1.0 / N;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        loss[0] = sl[0] / N;
        loss[1] = inv_n;
    }
    const int el = threadIdx.x % kFinalEntries, grp = threadIdx.x / kFinalEntries;
    const int k = blockIdx.x * kFinalEntries + el;
    const bool live = k < 3 * (kWPack + kC);
    const int layer = live ? k / (kWPack + kC) : 0, idx = k - layer * (kWPack + kC);
    const int per = (nparts + kFinalGroups - 1) / kFinalGroups;
    const int p0 = grp * per, p1 = min(nparts, p0 + per);
    float a = 0.f;
    if (live) {
        const float *src = parts + int64_t(layer) * nparts * (kWPack + kC) + idx;
        int p = p0;
        for (; p + 8 <= p1; p += 8) {
            float q[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) q[e] = src[int64_t(p + e) * (kWPack + kC)];
#pragma unroll
            for (int e = 0; e < 8; ++e) a += q[e];
        }
        for (; p < p1; ++p) a += src[int64_t(p) * (kWPack + kC)];
    }
    sg[grp][el] = a;
    __syncthreads();
    if (grp != 0 || !live) return;
    float sum = sg[0][el];
    for (int q = 1; q < kFinalGroups; ++q) sum += sg[q][el];
    sum = float(double(sum) * inv_n);
    const int cout = layer == 2 ? 1 : 16, cin = layer == 0 ? 2 : 16;
    const int wbase = layer == 0 ? kW1 : (layer == 1 ? kW2 : kW3);
    const int bbase = layer == 0 ? kB1 : (layer == 1 ? kB2 : kB3);
    if (idx < kWPack) {
        const int t = idx / (kC * kC), co = (idx / kC) % kC, ci = idx % kC;
        if (co < cout && ci < cin) grad[wbase + (co * cin + ci) * kTaps + t] = sum;
    } else {
        const int co = idx - kWPack;
        if (co < cout) grad[bbase + co] = sum;
    }
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


static inline unsigned grid1(int64_t n, int bs = 256) { return unsigned((n + bs - 1) / bs); }


// ---------------------------------------------------------------------------
// Fused inference: gather, three layers and the warm-start epilogue of one
// tile per iteration of a workgroup, activations in LDS only.  Every layer
// is an implicit GEMM on v_mfma_f32_16x16x32_bf16 (16 voxels x 16 output
// channels x 32 products of (tap, input channel)); the weights of all three
// layers stay in registers for the whole launch.

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

constexpr int kL1M = 3;       // layer 1: per lane group a (y, z) tap pair, its 3 x taps + 1 zero slot x 2 channels
constexpr int kL2M = 14;      // layer 2: 27 taps x 16 channels, two taps per MFMA
constexpr int kL3M = 2;       // layer 3: rows = the 9 (y, z) tap pairs, K = 3 x taps x 16 channels
// layer 1 runs on the weight pair hi + lo (bfloat16(W) and bfloat16(W -
// bfloat16(W))): its few input channels make the layer's output sensitive to
// the rounding of W1, and the second MFMA per K step costs little
constexpr int kLaneW = (2 * kL1M + kL2M + kL3M) * 64 * 8;

// The workspace of one network call (caller device memory): packed
// weights, activations of n tiles and, for training, their gradients and
// the weight-gradient partial sums.
struct NetWS {
    // forward (dn_net_forward)
    uint16_t *wpack, *x0, *h1, *h2;
    float *r;
    // training step (dn_net_loss_grad)
    uint16_t *lanew, *lanef, *gates, *x1cf, *h1cf, *h2cf, *d3cf, *d2cf, *d1cf;
    float *rc, *d3, *parts;
    double *misc, *tl, *tc;
    int nparts;
};
constexpr int kMaxWgradGroups = 256;
static NetWS carve_net(Bump &b, int64_t n, bool training)
{
    NetWS x{};
    if (!training) {
        const size_t act = size_t(n) * kT * kC;
        x.wpack = b.take<uint16_t>(size_t(4) * kWPack);
        x.x0 = b.take<uint16_t>(act);
        x.h1 = b.take<uint16_t>(act);
        x.h2 = b.take<uint16_t>(act);
        x.r = b.take<float>(size_t(n) * kT);
        return x;
    }
    x.lanew = b.take<uint16_t>(size_t(kLaneW));
    x.lanef = b.take<uint16_t>(size_t(kL2M) * 64 * 8);
    x.gates = b.take<uint16_t>(size_t(n) * 2 * kT);
    x.x1cf = b.take<uint16_t>(size_t(n) * 2 * kPadVox);
    x.h1cf = b.take<uint16_t>(size_t(n) * 16 * kPadVox);
    x.h2cf = b.take<uint16_t>(size_t(n) * 16 * kPadVox);
    x.rc = b.take<float>(size_t(n) * kBlockVox);
    x.d3 = b.take<float>(size_t(n) * kBlockVox);
    x.d3cf = b.take<uint16_t>(size_t(n) * kRowVox);
    x.d2cf = b.take<uint16_t>(size_t(n) * 16 * kRowVox);
    x.d1cf = b.take<uint16_t>(size_t(n) * 16 * kRowVox);
    x.nparts = int(n < kMaxWgradGroups ? n : kMaxWgradGroups);
    x.parts = b.take<float>(size_t(3) * x.nparts * (kWPack + kC));
    x.misc = b.take<double>(8);
    x.tl = b.take<double>(size_t(n));
    x.tc = b.take<double>(size_t(n));
    return x;
}

static bool ws_ok(const void *ws) { return ws && (reinterpret_cast<uintptr_t>(ws) & 255) == 0; }

// Lane-ready weights [mfma][lane][8] (bfloat16).  The K slots of lane
// group g = lane / 16, entry j, of MFMA m: layer 1 -> tap 16m + 4g + j/2,
// channel j%2; layer 2 -> tap 2m + g/2, channel 8(g%2) + j; the output
// column (output channel) is lane % 16.  Layer 3 has one output channel, so
// its rows are taps instead: row n = 3 kz + ky (n < 9) is the (y, z) tap
// pair, and the K slots of MFMA m, group g are x tap kx = 2m + g/2 (kx < 3),
// channel 8(g%2) + j.  The activation operand uses the same map, so the
// products pair up whatever order the hardware sums them in.
__device__ void pack_lane(const float *__restrict__ params, int k, uint16_t *__restrict__ out)
{
    const int j = k & 7, lane = (k >> 3) & 63, m = k >> 9;
    const int g = lane >> 4, n = lane & 15;
    float val = 0.f;
    if (m < kL1M || m >= kL1M + kL2M + kL3M) {
        const int ml = m < kL1M ? m : m - (kL1M + kL2M + kL3M);
        const int pr = 4 * ml + g, e = j >> 1, ci = j & 1;   // (y, z) pair, x slot, channel
        if (pr < 9 && e < 3) val = params[kW1 + (n * 2 + ci) * kTaps + e + 3 * pr];
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

__global__ void k_pack_lanes(const float *__restrict__ params, uint16_t *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kLaneW) pack_lane(params, k, out);
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
//
// kTrain: the forward pass of a training step on n given tiles (f holds the
// float tiles [n][2][1000]); the layer inputs are also written to global
// memory on the zero-padded 12^3 grid for the backward pass (x1cf: the two
// input channels channel-first, [n][2][1728]; h1cf, h2cf channel-last,
// [n][1728][16]), and out receives the residual r on the centre, [n][512]
// (voxel x + 8y + 64z).
__device__ __forceinline__ int pad_index(int x, int y, int z) { return (x + 1) + 12 * (y + 1) + 144 * (z + 1); }

// Channel-last copy of an LDS activation (two planes of 8 channels) onto the
// padded grid: dst[1728][16], 32 bytes per padded voxel, zero on the padding.
__device__ __forceinline__ void copy_act_cl(const uint16_t *h, uint16_t *__restrict__ dst, int tid)
{
    for (int p = tid; p < kPadVox; p += 256) {
        const int x = p % 12 - 1, y = (p / 12) % 12 - 1, z = p / 144 - 1;
        uint4 lo = make_uint4(0, 0, 0, 0), hi = lo;
        if (x >= 0 && x < 10 && y >= 0 && y < 10 && z >= 0 && z < 10) {
            const int v = x + 10 * y + 100 * z;
            lo = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(h) + act_byte(v, 0));
            hi = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(h) + act_byte(v, 1));
        }
        reinterpret_cast<uint4 *>(dst)[2 * p] = lo;
        reinterpret_cast<uint4 *>(dst)[2 * p + 1] = hi;
    }
}

// Bit ch of dst[v] set when channel ch of the LDS activation is positive at
// tile voxel v (the open ReLUs the backward pass gates with).
__device__ __forceinline__ void gate_bits(const uint16_t *h, uint16_t *__restrict__ dst, int tid)
{
    for (int v = tid; v < kT; v += 256) {
        const uint4 lo = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(h) + act_byte(v, 0));
        const uint4 hi = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(h) + act_byte(v, 1));
        const uint32_t w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
        uint32_t m = 0;
        for (int k = 0; k < 8; ++k) {
            const uint32_t a = w[k] & 0xFFFFu, c = w[k] >> 16;
            if (!(a & 0x8000u) && (a & 0x7FFFu)) m |= 1u << (2 * k);
            if (!(c & 0x8000u) && (c & 0x7FFFu)) m |= 1u << (2 * k + 1);
        }
        dst[v] = uint16_t(m);
    }
}

template <bool kTrain>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_net_fwd(
    const int32_t *__restrict__ nbr, const uint32_t *__restrict__ pair, const float *__restrict__ f,
    const uint8_t *__restrict__ emask, int64_t nb, int perm, int mode, const uint16_t *__restrict__ lw,
    const float *__restrict__ params, int64_t ps, float *__restrict__ out, uint16_t *__restrict__ x1cf,
    uint16_t *__restrict__ h1cf, uint16_t *__restrict__ h2cf, uint16_t *__restrict__ gates)
{
    __shared__ __align__(16) uint16_t h1[2 * kPlane / 2];
    __shared__ __align__(16) uint16_t h2[2 * kPlane / 2];
    __shared__ __align__(16) uint32_t x0[kPadVox + 4];   // layer-1 input words on the zero-bordered 12^3 grid
                                                        // (+ the last x slot of the last voxel)
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
    for (int k = tid; k < kPadVox + 4; k += 256) x0[k] = 0u;

    // the layer-1 input of a tile, read from the pool's pair words through
    // the neighbour table (tile voxels of unallocated blocks give 0), the
    // next tile's while this one is computed
    constexpr int kGet = (kT + 255) / 256;
    uint32_t nxt[kGet];
    auto fetch = [&](int64_t bb) {
        if constexpr (kTrain) {
            // the tiles are float [n][2][1000] (f, then the weight channel)
            for (int e = 0; e < kGet; ++e) {
                const int k = tid + 256 * e;
                nxt[e] = k < kT ? (uint32_t(f2bf(f[bb * 2 * kT + k])) | (uint32_t(f2bf(f[bb * 2 * kT + kT + k])) << 16))
                                : 0u;
            }
            return;
        }
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
            if (tid + 256 * e < kT) {
                const int k = tid + 256 * e;
                x0[pad_index(k % 10, (k / 10) % 10, k / 100)] = nxt[e];
            }
        __syncthreads();
        const int64_t bn = b + gridDim.x;
        if (bn < nb) fetch(bn);

        // layer 1: 2 -> 16, ReLU.  Lane group g of MFMA m takes the (y, z)
        // tap pair 4m + g: the input words of its x taps -1, 0, +1 (and +2,
        // whose weights are zero) are 4 consecutive words of the padded
        // grid, zero wherever the tap leaves the tile.
        for (int mt = wave; mt < kMT; mt += 4) {
            const int v = vt[mt * 16 + i];
            const int pv = v < kT ? pad_index(v % 10, (v / 10) % 10, v / 100) : pad_index(0, 0, 0);
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            for (int m = 0; m < kL1M; ++m) {
                const int pr = 4 * m + g;
                const int at = pr < 9 ? pv - 1 + 12 * (pr % 3 - 1) + 144 * (pr / 3 - 1) : 0;
                const v4u q = {x0[at], x0[at + 1], x0[at + 2], x0[at + 3]};
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W1[m], as_v8bf(q), acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W1l[m], as_v8bf(q), acc, 0, 0, 0);
            }
            store_act(h1, v, g, acc, bias1);
        }
        __syncthreads();
        if constexpr (kTrain) {
            // layer inputs for the backward pass (read-only use of h1 and x0
            // until the barrier after layer 2), and which ReLUs are open
            copy_act_cl(h1, h1cf + b * (16 * kPadVox), tid);
            gate_bits(h1, gates + b * (2 * kT), tid);
            for (int e = tid; e < 2 * kPadVox; e += 256) {
                const int ch = e / kPadVox, p = e - ch * kPadVox;
                x1cf[b * (2 * kPadVox) + e] = uint16_t(x0[p] >> (16 * ch));
            }
        }

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
        if constexpr (kTrain) {
            copy_act_cl(h2, h2cf + b * (16 * kPadVox), tid);
            gate_bits(h2, gates + b * (2 * kT) + kT, tid);
        }

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
            const float rv = acc + bias3;
            if constexpr (kTrain) {
                out[b * kBlockVox + c] = rv;
                continue;
            }
            int x = cx, y = cy, z = cz;
            if (perm == 1) { const int sw = x; x = y; y = sw; }
            if (perm == 2) { const int sw = x; x = z; z = sw; }
            const int64_t gi = b * kBlockVox + x + 8 * y + 64 * z;
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

// ---------------------------------------------------------------------------
// Training step kernels (after k_net_fwd<true>).

// Lane-ready weights of a training step: the forward's (as k_pack_lanes)
// and those of the input gradient of layer 2, d1 = conv(d2, W') with
// W'[ci][co][t] = W2[co][ci][26 - t] (the layer-2 map of k_pack_lanes).
__device__ void pack_lane(const float *__restrict__ params, int k, uint16_t *__restrict__ out);
__global__ void k_pack_train(const float *__restrict__ params, uint16_t *__restrict__ lw, uint16_t *__restrict__ out)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kLaneW) {
        pack_lane(params, k, lw);
        return;
    }
    k -= kLaneW;
    if (k >= kL2M * 64 * 8) return;
    const int j = k & 7, lane = (k >> 3) & 63, m = k >> 9;
    const int g = lane >> 4, n = lane & 15;
    const int t = 2 * m + (g >> 1), c = 8 * (g & 1) + j;
    float val = 0.f;
    if (t < kTaps) val = params[kW2 + (c * 16 + n) * kTaps + (kTaps - 1 - t)];
    out[k] = f2bf(val);
}

__device__ __forceinline__ bool bf_pos(uint16_t h) { return !(h & 0x8000u) && (h & 0x7FFFu) != 0; }

// Compact-row index of tile voxel (x, y, z), and its decoding (false for
// padding entries).
__device__ __forceinline__ int row_index(int x, int y, int z) { return (x + 1) + 12 * (10 * z + y); }
__device__ __forceinline__ bool row_voxel(int c, int &x, int &y, int &z)
{
    if (c >= 1200) return false;
    const int xr = c % 12, r = c / 12;
    x = xr - 1; y = r % 10; z = r / 10;
    return xr >= 1 && xr <= 10;
}

// Masked squared loss of one tile per workgroup (512 threads, one per
// centre voxel), before the division by N = max(1, sum of the mask), which
// k_grad_final forms and applies: d3 = N dL/dr on the centre
// (float [n][512]) and the same in the compact-row layout for the weight
// gradient of layer 3 (d3cf [n][1216], bfloat16, zero off the centre), the
// tile's sum of squared errors and of the mask.
__global__ __launch_bounds__(512) void k_loss_train(const float *__restrict__ tiles, const float *__restrict__ R,
                                                    const float *__restrict__ targets, const float *__restrict__ mask,
                                                    int64_t n, int kind, float *__restrict__ d3,
                                                    uint16_t *__restrict__ d3cf, double *__restrict__ tile_loss,
                                                    double *__restrict__ tile_count)
{
    __shared__ double sl[8], sc[8];
    __shared__ uint16_t sg[kT];
    const int64_t tile = blockIdx.x;
    const int v = threadIdx.x;
    const int cx = v & 7, cy = (v >> 3) & 7, cz = v >> 6;
    const int tv = (cx + 1) + 10 * (cy + 1) + 100 * (cz + 1);
    const double m = mask[tile * 512 + v];
    const double e = (kind == 0 ? double(tiles[tile * 2 * kT + tv]) : 0.0) + double(R[tile * 512 + v]) -
                     double(targets[tile * 512 + v]);
    double l = m != 0.0 ? e * e : 0.0, c = m;
    const float gv = m != 0.0 ? float(2.0 * e) : 0.f;
    d3[tile * 512 + v] = gv;
    for (int k = v; k < kT; k += 512) sg[k] = 0;
    __syncthreads();
    sg[tv] = f2bf(gv);
    for (int o = 32; o > 0; o >>= 1) {
        l += __shfl_xor(l, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    if ((v & 63) == 0) {
        sl[v >> 6] = l;
        sc[v >> 6] = c;
    }
    __syncthreads();
    uint16_t *dst = d3cf + tile * kRowVox;
    for (int k = v; k < kRowVox; k += 512) {
        uint16_t val = 0;
        int x, y, z;
        if (row_voxel(k, x, y, z)) val = sg[x + 10 * y + 100 * z];
        dst[k] = val;
    }
    if (v == 0) {
        double s = 0.0, t = 0.0;
        for (int k = 0; k < 8; ++k) {
            s += sl[k];
            t += sc[k];
        }
        tile_loss[tile] = s;
        tile_count[tile] = t;
    }
}

// Backward through layers 3 and 2 of one tile per iteration of a
// workgroup, on MFMA: d2 = (W3 applied backwards to d3) gated by [h2 > 0],
// as one 16 (channels) x 16 (voxels) x 32 (taps) product per row tile (the
// lane's 8 taps read d3 shifted back by the tap), then d1 = conv(d2, W')
// gated by [h1 > 0] as layer 2 of k_net_fwd (flipped weights W' in
// registers, d2 in LDS).  d2 and d1 go to global memory on the compact
// rows, channel-last ([n][1216][16] bfloat16, 32 bytes per entry).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_net_bwd(
    const float *__restrict__ d3, const uint16_t *__restrict__ gates, int64_t n, const uint16_t *__restrict__ lwf,
    const float *__restrict__ params, uint16_t *__restrict__ d2cf, uint16_t *__restrict__ d1cf)
{
    __shared__ __align__(16) uint16_t dd[2 * kPlane / 2];
    __shared__ uint16_t s3[kT + 8];          // d3 on the tile (bfloat16; entry kT stays zero)
    __shared__ __align__(16) uint16_t sg[2 * kT];    // open ReLUs of layers 1 and 2 (bit = channel)
    __shared__ uint32_t okt[kMT * 16];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int v = tid; v < kMT * 16; v += 256) okt[v] = v < kT ? tap_mask(v % 10, (v / 10) % 10, v / 100) : 0u;
    for (int v = tid; v < kT + 8; v += 256) s3[v] = 0;
    const int i = lane & 15, g = lane >> 4;
    const int half = g & 1, par = g >> 1;
    const v4u *lw4 = reinterpret_cast<const v4u *>(lwf);
    v8bf W2[kL2M];
    for (int m = 0; m < kL2M; ++m) W2[m] = as_v8bf(lw4[m * 64 + lane]);
    // W3 as the first operand: row ci = i, K slots = taps 8g .. 8g + 7
    v8bf W3r;
    {
        uint16_t w[8];
        for (int j = 0; j < 8; ++j) {
            const int t = 8 * g + j;
            w[j] = t < kTaps ? f2bf(params[kW3 + i * kTaps + t]) : uint16_t(0);
        }
        W3r = as_v8bf(*reinterpret_cast<const v4u *>(&w[0]));
    }
    int toff[8];
    for (int j = 0; j < 8; ++j) {
        const int t = 8 * g + j;
        toff[j] = t < kTaps ? tap_off(t) : 0;
    }
    if (tid < 8) reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(dd) + (tid >> 2) * kPlane + kT * 16)[tid & 3] = 0u;
    // the next tile's d3 (2 centre values per thread) and gate words (one
    // 16-byte chunk per thread) are loaded while the current one is computed
    float2 nd3 = make_float2(0.f, 0.f);
    uint4 ngt = make_uint4(0, 0, 0, 0);
    auto fetch = [&](int64_t bb) {
        nd3 = reinterpret_cast<const float2 *>(d3 + bb * 512)[tid];
        if (tid < 2 * kT / 8) ngt = reinterpret_cast<const uint4 *>(gates + bb * (2 * kT))[tid];
    };
    if (blockIdx.x < n) fetch(blockIdx.x);
    __syncthreads();
    for (int64_t b = blockIdx.x; b < n; b += gridDim.x) {
        {
            const int c0 = 2 * tid;       // centre voxels c0, c0 + 1 (same x row)
            const int cx = c0 & 7, cy = (c0 >> 3) & 7, cz = c0 >> 6;
            const int v = (cx + 1) + 10 * (cy + 1) + 100 * (cz + 1);
            s3[v] = f2bf(nd3.x);
            s3[v + 1] = f2bf(nd3.y);
            if (tid < 2 * kT / 8) reinterpret_cast<uint4 *>(sg)[tid] = ngt;
        }
        const int64_t bn = b + gridDim.x;
        if (bn < n) fetch(bn);
        __syncthreads();
        uint16_t *o2 = d2cf + b * (16 * kRowVox);
        uint16_t *o1 = d1cf + b * (16 * kRowVox);
        // d2 = W3^T d3 (shifted back), gated by [h2 > 0]
        for (int mt = wave; mt < kMT; mt += 4) {
            const int v = mt * 16 + i;
            const uint32_t ok = okt[v < kT ? v : kT];
            uint16_t q[8];
            for (int j = 0; j < 8; ++j) {
                const int t = 8 * g + j;
                // d3 at v - off(t): inside the tile when tap 26 - t of v is
                q[j] = s3[(t < kTaps && ((ok >> (kTaps - 1 - t)) & 1u)) ? v - toff[j] : kT];
            }
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W3r, as_v8bf(*reinterpret_cast<const v4u *>(&q[0])), acc,
                                                         0, 0, 0);
            if (v < kT) {
                // lane: voxel v, channels 4g .. 4g + 3
                const uint32_t open2 = sg[kT + v];
                uint16_t r4[4];
                for (int r = 0; r < 4; ++r) r4[r] = ((open2 >> (4 * g + r)) & 1u) ? f2bf(acc[r]) : uint16_t(0);
                const uint2 pk = *reinterpret_cast<const uint2 *>(&r4[0]);
                *reinterpret_cast<uint2 *>(reinterpret_cast<char *>(dd) + act_byte(v, g >> 1) + 8 * (g & 1)) = pk;
                const int x = v % 10, y = (v / 10) % 10, z = v / 100;
                reinterpret_cast<uint2 *>(o2 + row_index(x, y, z) * 16)[g] = pk;
            }
        }
        for (int c = tid; c < kRowVox; c += 256) {
            int x, y, z;
            if (!row_voxel(c, x, y, z)) {
                reinterpret_cast<uint4 *>(o2)[2 * c] = make_uint4(0, 0, 0, 0);
                reinterpret_cast<uint4 *>(o2)[2 * c + 1] = make_uint4(0, 0, 0, 0);
                reinterpret_cast<uint4 *>(o1)[2 * c] = make_uint4(0, 0, 0, 0);
                reinterpret_cast<uint4 *>(o1)[2 * c + 1] = make_uint4(0, 0, 0, 0);
            }
        }
        __syncthreads();
        // d1 = conv(d2, W') gated by [h1 > 0]
        for (int mt = wave; mt < kMT; mt += 4) {
            const int v = mt * 16 + i;
            const uint32_t ok = okt[v < kT ? v : kT];
            const v4f acc = mfma_chain<kL2M, 5, false>(
                [&](int m) {
                    const int o = par ? tap_off(2 * m + 1) : tap_off(2 * m);
                    const int nv = ((ok >> (2 * m + par)) & 1u) ? v + o : kT;
                    return as_v8bf(lds_row(dd, act_byte(nv, half)));
                },
                [&](int m) { return W2[m]; });
            if (v < kT) {
                const int x = v % 10, y = (v / 10) % 10, z = v / 100;
                const int c = row_index(x, y, z);
                const uint32_t open1 = sg[v];
                uint16_t q[4];
                for (int r = 0; r < 4; ++r) q[r] = ((open1 >> (4 * g + r)) & 1u) ? f2bf(acc[r]) : uint16_t(0);
                reinterpret_cast<uint2 *>(o1 + c * 16)[g] = *reinterpret_cast<const uint2 *>(&q[0]);
            }
        }
        // d3 entries back to zero for the next tile
        {
            const int c0 = 2 * tid;
            const int cx = c0 & 7, cy = (c0 >> 3) & 7, cz = c0 >> 6;
            const int v = (cx + 1) + 10 * (cy + 1) + 100 * (cz + 1);
            s3[v] = 0;
            s3[v + 1] = 0;
        }
        __syncthreads();
    }
}

// LDS rows: X channel rows of 1928 entries (8 + 1728 + zero margin; 964
// words, 4 modulo 64 banks, so the 16 lanes of a 16-byte read start on 16
// distinct groups of 4 banks), dY rows of 1224 entries (612 words, 36 modulo
// 64, likewise).
constexpr int kXRow = 1928;
constexpr int kDRow = 1224;

// Eight channel values (one 16-byte chunk of a channel-last entry) into
// eight channel rows of an LDS tile: row0[j * stride + pos] = channel j.
__device__ __forceinline__ void scatter8(uint16_t *row0, int stride, int pos, uint4 v)
{
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        row0[(2 * j) * stride + pos] = uint16_t(w[j] & 0xFFFFu);
        row0[(2 * j + 1) * stride + pos] = uint16_t(w[j] >> 16);
    }
}

// The three x shifts of a run of 8 channel-row entries starting at p
// (p 8-byte aligned): bm = p[-1 .. 6], b0 = p[0 .. 7], bp = p[1 .. 8], from
// four aligned 8-byte reads of p[-4 .. 11] and 16-bit funnel shifts (an
// LDS read at a 2-byte offset is split by the hardware and costs several
// times an aligned one).
__device__ __forceinline__ void x_shifts(const uint16_t *p, v4u &bm, v4u &b0, v4u &bp)
{
    const uint2 *q = reinterpret_cast<const uint2 *>(p - 4);
    const uint2 l0 = q[0], l1 = q[1], l2 = q[2], l3 = q[3];
    const uint32_t s1 = __builtin_amdgcn_alignbit(l1.y, l1.x, 16), s2 = __builtin_amdgcn_alignbit(l2.x, l1.y, 16),
                   s3 = __builtin_amdgcn_alignbit(l2.y, l2.x, 16);
    bm = v4u{__builtin_amdgcn_alignbit(l1.x, l0.y, 16), s1, s2, s3};
    b0 = v4u{l1.x, l1.y, l2.x, l2.y};
    bp = v4u{s1, s2, s3, __builtin_amdgcn_alignbit(l3.x, l2.y, 16)};
}

// The shift s in {-1, 0, +1} of that run (p[s .. s + 7]), s per lane.
__device__ __forceinline__ v4u x_shift(const uint16_t *p, int s)
{
    v4u bm, b0, bp;
    x_shifts(p, bm, b0, bp);
    return s < 0 ? bm : (s > 0 ? bp : b0);
}

// Eight entries p[0 .. 7] at an 8-byte aligned p, as two aligned reads.
__device__ __forceinline__ v4u lds8_a8(const uint16_t *p)
{
    const uint2 *q = reinterpret_cast<const uint2 *>(p);
    const uint2 l1 = q[0], l2 = q[1];
    return v4u{l1.x, l1.y, l2.x, l2.y};
}

// Weight and bias gradient of layer 3 (one output channel):
//   dW3[ci][t] = sum over tile voxels v of h2[ci][v] d3[v - off(t)],
// as (taps, 16 rows) x (input channels, 16 columns) x (32 voxels) MFMAs:
// the rows read d3, kept on the padded grid, shifted back by their own tap
// (x shifts per lane from x_shift), the columns read h2 unshifted.  Two MFMAs per
// 32 voxels instead of 27 with one used row.  Partials in the
// [tap][co][ci] layout (co = 0), bias db3 = sum of d3.
constexpr int kD3Row = 2080;   // LDS entries of d3: 168 zero margin + 1728 + margin
constexpr int kWgrad3Lds = 2 * 16 * kXRow + 2 * kD3Row + 4 * 256 + 4 * 4 * 32 * 16;
__device__ __forceinline__ void wgrad3_body(const uint16_t *__restrict__ X, const uint16_t *__restrict__ d3cf,
                                            int64_t n, float *__restrict__ partials, int wg, int ngroups,
                                            uint8_t *lds)
{
    uint16_t *sx = reinterpret_cast<uint16_t *>(lds);                  // [16][kXRow]
    uint16_t *sd = sx + 16 * kXRow;                                     // [kD3Row]
    float *sb = reinterpret_cast<float *>(sd + kD3Row);                 // [256]
    float(*red)[32][16] = reinterpret_cast<float(*)[32][16]>(sb + 256);  // [4][32][16]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i = lane & 15, g = lane >> 4;
    for (int k = tid; k < 16 * kXRow / 8; k += 256) reinterpret_cast<uint4 *>(sx)[k] = make_uint4(0, 0, 0, 0);
    for (int k = tid; k < kD3Row / 8; k += 256) reinterpret_cast<uint4 *>(sd)[k] = make_uint4(0, 0, 0, 0);
    v4f acc[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
    float bsum = 0.f;
    __syncthreads();
    constexpr int kXc = kPadVox / 8;
    constexpr int kPer = (16 * kXc + 255) / 256;
    constexpr int kDPer = (kRowVox + 255) / 256;
    uint4 nxt[kPer];
    uint16_t nd[kDPer];
    auto fetch = [&](int64_t tl) {
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int k = tid + 256 * e;
            if (k < 16 * kXc) nxt[e] = reinterpret_cast<const uint4 *>(X + tl * 16 * kPadVox)[k];
        }
#pragma unroll
        for (int e = 0; e < kDPer; ++e) {
            const int c = tid + 256 * e;
            nd[e] = c < kRowVox ? d3cf[tl * kRowVox + c] : uint16_t(0);
        }
    };
    if (wg < n) fetch(wg);
    for (int64_t tile = wg; tile < n; tile += ngroups) {
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int k = tid + 256 * e;
            if (k < 16 * kXc) scatter8(sx + (k & 1) * 8 * kXRow + 8, kXRow, k >> 1, nxt[e]);
        }
        // d3 from its compact rows onto the padded grid (zero elsewhere)
#pragma unroll
        for (int e = 0; e < kDPer; ++e) {
            const int c = tid + 256 * e;
            int x, y, z;
            if (c < kRowVox && row_voxel(c, x, y, z)) {
                sd[168 + pad_index(x, y, z)] = nd[e];
                bsum += bf2f(nd[e]);
            }
        }
        __syncthreads();
        if (tile + ngroups < n) fetch(tile + ngroups);
        // wave w takes the 32-voxel chunks w, w + 4, ...
        for (int c0 = 32 * wave; c0 < kRowVox; c0 += 128) {
            const int c = c0 + 8 * g;
            const int plane = c / 120, within = c - 120 * plane;
            const int pc = within + 12 + 144 * (plane + 1);          // padded index of entry c
            const v8bf b = as_v8bf(lds8_a8(sx + i * kXRow + 8 + pc));
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = 16 * h + i;
                v4u q = {0u, 0u, 0u, 0u};
                if (t < kTaps)
                    q = x_shift(sd + 168 + pc - 12 * ((t / 3) % 3 - 1) - 144 * (t / 9 - 1), 1 - t % 3);
                acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_v8bf(q), b, acc[h], 0, 0, 0);
            }
        }
        __syncthreads();
        for (int c = tid; c < kRowVox; c += 256) {      // clear d3's entries for the next tile
            int x, y, z;
            if (row_voxel(c, x, y, z)) sd[168 + pad_index(x, y, z)] = 0;
        }
    }
    // the four waves' sums of each (tap, ci), then one partial per workgroup
    for (int h = 0; h < 2; ++h)
        for (int r = 0; r < 4; ++r) red[wave][16 * h + 4 * g + r][i] = acc[h][r];
    sb[tid] = bsum;
    __syncthreads();
    float *out = partials + int64_t(wg) * (kWPack + kC);
    for (int e = tid; e < kWPack + kC; e += 256) {
        float v = 0.f;
        if (e < kWPack) {
            const int t = e / (kC * kC), co = (e / kC) % kC, ci = e % kC;
            if (co == 0) v = ((red[0][t][ci] + red[1][t][ci]) + red[2][t][ci]) + red[3][t][ci];
        } else if (e == kWPack) {
            for (int k = 0; k < 256; ++k) v += sb[k];
        }
        out[e] = v;
    }
}

// Weight and bias gradient of layer 1 (two input channels):
//   dW1[co][ci][t] = sum over v of d1[co][v] x[ci][v + off(t)],
// as (output channels) x (54 (ci, t) columns in four MFMAs) x (32 voxels):
// each column reads the input channel shifted by its own tap (the y and z
// shifts keep the reads 8-byte aligned, x shifts per lane from x_shift).
constexpr int kWgrad1Lds = 2 * 2 * kXRow + 2 * 16 * kDRow + 4 * 256 + 4 * 4 * 16 * 64;
__device__ __forceinline__ void wgrad1_body(const uint16_t *__restrict__ X, const uint16_t *__restrict__ dY,
                                            int64_t n, float *__restrict__ partials, int wg, int ngroups,
                                            uint8_t *lds)
{
    uint16_t *sx = reinterpret_cast<uint16_t *>(lds);                  // [2][kXRow]
    uint16_t *sd = sx + 2 * kXRow;                                      // [16][kDRow]
    float *sb = reinterpret_cast<float *>(sd + 16 * kDRow);             // [256]
    float(*red)[16][64] = reinterpret_cast<float(*)[16][64]>(sb + 256);  // [4][16][64]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i = lane & 15, g = lane >> 4;
    for (int k = tid; k < 2 * kXRow / 8; k += 256) reinterpret_cast<uint4 *>(sx)[k] = make_uint4(0, 0, 0, 0);
    for (int k = tid; k < 16 * kDRow / 8; k += 256) reinterpret_cast<uint4 *>(sd)[k] = make_uint4(0, 0, 0, 0);
    v4f acc[4];
    for (int q = 0; q < 4; ++q) acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    int coff[4], ckx[4];             // column 16 q + i: channel row + (y, z) tap shift, and its x shift
    bool cuse[4];
    for (int q = 0; q < 4; ++q) {
        const int col = 16 * q + i, ci = col / kTaps, t = col % kTaps;
        cuse[q] = col < 2 * kTaps;
        coff[q] = cuse[q] ? ci * kXRow + 8 + 12 * ((t / 3) % 3 - 1) + 144 * (t / 9 - 1) : 8;
        ckx[q] = t % 3 - 1;
    }
    __syncthreads();
    constexpr int kXc = kPadVox / 8, kDc = kRowVox / 8;
    constexpr int kChunks = 2 * kXc + 16 * kDc;
    constexpr int kPer = (kChunks + 255) / 256;
    uint4 nxt[kPer];
    auto fetch = [&](int64_t tl) {
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int k = tid + 256 * e;
            if (k < 2 * kXc) nxt[e] = reinterpret_cast<const uint4 *>(X + tl * 2 * kPadVox)[k];
            else if (k < kChunks) nxt[e] = reinterpret_cast<const uint4 *>(dY + tl * 16 * kRowVox)[k - 2 * kXc];
        }
    };
    if (wg < n) fetch(wg);
    for (int64_t tile = wg; tile < n; tile += ngroups) {
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int k = tid + 256 * e;
            if (k < 2 * kXc) {
                const int ch = k / kXc, r = k - ch * kXc;
                reinterpret_cast<uint4 *>(sx + ch * kXRow + 8)[r] = nxt[e];
            } else if (k < kChunks) {
                const int kk = k - 2 * kXc;
                scatter8(sd + (kk & 1) * 8 * kDRow, kDRow, kk >> 1, nxt[e]);
            }
        }
        __syncthreads();
        if (tile + ngroups < n) fetch(tile + ngroups);
        for (int c = tid >> 4; c < kRowVox; c += 16) bsum += bf2f(sd[(tid & 15) * kDRow + c]);
        for (int c0 = 32 * wave; c0 < kRowVox; c0 += 128) {
            const int c = c0 + 8 * g;
            const v8bf a = as_v8bf(*reinterpret_cast<const v4u *>(sd + i * kDRow + c));
            const int plane = c / 120, within = c - 120 * plane;
            const int pc = within + 12 + 144 * (plane + 1);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v4u bq = {0u, 0u, 0u, 0u};
                if (cuse[q]) bq = x_shift(sx + coff[q] + pc, ckx[q]);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, as_v8bf(bq), acc[q], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // D[co][col]: lane holds column 16 q + i, rows co = 4g .. 4g + 3; the
    // four waves' sums, then one partial per workgroup in [tap][co][ci]
    for (int q = 0; q < 4; ++q)
        for (int r = 0; r < 4; ++r) red[wave][4 * g + r][16 * q + i] = acc[q][r];
    sb[tid] = bsum;
    __syncthreads();
    float *out = partials + int64_t(wg) * (kWPack + kC);
    for (int e = tid; e < kWPack + kC; e += 256) {
        float v = 0.f;
        if (e < kWPack) {
            const int t = e / (kC * kC), co = (e / kC) % kC, ci = e % kC;
            if (ci < 2) {
                const int col = ci * kTaps + t;
                v = ((red[0][co][col] + red[1][co][col]) + red[2][co][col]) + red[3][co][col];
            }
        } else {
            const int co = e - kWPack;
            for (int k = 0; k < 16; ++k) v += sb[k * 16 + co];
        }
        out[e] = v;
    }
}

// The layer-1 and layer-3 weight gradients in one launch: workgroups
// [0, g1) take layer 1, the rest layer 3.  Each is latency-bound with one
// workgroup per compute unit; sharing one LDS allocation (the larger of the
// two) lets a unit hold one of each, so the two run side by side.
constexpr int kWgrad13Lds = kWgrad1Lds > kWgrad3Lds ? kWgrad1Lds : kWgrad3Lds;
__global__ __launch_bounds__(256) void k_wgrad13(const uint16_t *__restrict__ X1, const uint16_t *__restrict__ d1,
                                                 const uint16_t *__restrict__ X3, const uint16_t *__restrict__ d3,
                                                 int64_t n, float *__restrict__ parts1, float *__restrict__ parts3,
                                                 int g1)
{
    __shared__ __align__(16) uint8_t lds[kWgrad13Lds];
    const int wg = int(blockIdx.x);
    if (wg < g1) wgrad1_body(X1, d1, n, parts1, wg, g1, lds);
    else wgrad3_body(X3, d3, n, parts3, wg - g1, int(gridDim.x) - g1, lds);
}

// LDS rows of the layer-2 weight gradient.  Its X reads are 8-byte reads
// by 16 channel rows x 4 lane groups whose runs are 64 entries (32 banks)
// apart: a row stride of 2 banks modulo 64 (1924 entries) puts the 32 lanes
// of each half-wave pass on 64 distinct banks.  dY rows of 1288 entries (4
// banks modulo 64) keep its 16-byte reads conflict-free, and hold the 1280
// entries the K steps cover (the compact rows' 1216 and zeros).
constexpr int kXRow2 = 1924;
constexpr int kDRow2 = 1288;
constexpr int kRowVox2 = 1280;

// Weight and bias gradient of layer 2 on MFMA (X = h1 channel-last on the
// padded grid, dY = d2 channel-last on the compact rows, both turned
// channel-first as they enter LDS):
//   dW[co][ci][t] = sum over tile voxels v of dY[co][v] X[ci][v + off(t)],
//   db[co] = sum over v of dY[co][v],
// the products as 16 (co) x 16 (ci) x 32 (voxels) MFMAs: 32 consecutive
// compact-row entries of dY (aligned 16-byte reads) against the same
// entries of the padded X shifted by the tap (a run of 8 entries never
// leaves its z plane, where the two layouts are contiguous alike; the y and
// z shifts keep X 8-byte aligned, the x shifts come from x_shifts).  One
// workgroup per compute unit loops over tiles and keeps every tap's 16 x 16
// block in registers; one partial [27][16][16] + [16] per workgroup.
template <int CI, int CO>
__global__ __launch_bounds__(512) void k_wgrad_mfma(const uint16_t *__restrict__ X, const uint16_t *__restrict__ dY,
                                                    int64_t n, float *__restrict__ partials)
{
    __shared__ __align__(16) uint16_t sx[16 * kXRow2];
    __shared__ __align__(16) uint16_t sd[16 * kDRow2];
    __shared__ float sb[512];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i = lane & 15, g = lane >> 4;
    // wave w: the taps t = 3w .. 3w + 2 of the (y, z) offset pair w (x
    // offsets -1, 0, +1, one read for the three); waves 0..2 also tap
    // 24 + w of pair 8 (y and z offsets +1)
    const int ky = wave % 3 - 1, kz = wave / 3 - 1;
    for (int k = tid; k < 16 * kXRow2 / 8; k += 512) reinterpret_cast<uint4 *>(sx)[k] = make_uint4(0, 0, 0, 0);
    for (int k = tid; k < 16 * kDRow2 / 8; k += 512) reinterpret_cast<uint4 *>(sd)[k] = make_uint4(0, 0, 0, 0);
    v4f acc[4];
    for (int j = 0; j < 4; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    __syncthreads();
    // 16-byte chunks of a tile: X (CI channels) then dY (CO channels), the
    // next tile's held in registers while the current one is computed
    constexpr int kXc = kPadVox / 8, kDc = kRowVox / 8;
    constexpr int kChunks = CI * kXc + CO * kDc;
    constexpr int kPer = (kChunks + 511) / 512;
    uint4 nxt[kPer];
    auto fetch = [&](int64_t tl) {
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int k = tid + 512 * e;
            if (k < CI * kXc) nxt[e] = reinterpret_cast<const uint4 *>(X + tl * CI * kPadVox)[k];
            else if (k < kChunks) nxt[e] = reinterpret_cast<const uint4 *>(dY + tl * CO * kRowVox)[k - CI * kXc];
        }
    };
    if (blockIdx.x < n) fetch(blockIdx.x);
    for (int64_t tile = blockIdx.x; tile < n; tile += gridDim.x) {
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int k = tid + 512 * e;
            if (k < CI * kXc) {
                scatter8(sx + (k & 1) * 8 * kXRow2 + 8, kXRow2, k >> 1, nxt[e]);
            } else if (k < kChunks) {
                const int kk = k - CI * kXc;
                scatter8(sd + (kk & 1) * 8 * kDRow2, kDRow2, kk >> 1, nxt[e]);
            }
        }
        __syncthreads();
        if (tile + gridDim.x < n) fetch(tile + gridDim.x);
        for (int c = tid >> 4; c < kRowVox; c += 32) bsum += bf2f(sd[(tid & 15) * kDRow2 + c]);
        const uint16_t *xrow = sx + i * kXRow2;
        // K steps: runs of 8 entries 64 apart for the four lane groups
        // (c = cb + j + 64 g over 1280 entries, the last 64 zero in dY)
        for (int step = 0; step < kRowVox2 / 32; ++step) {
            const int c = 256 * (step >> 3) + 8 * (step & 7) + 64 * g;
            const v8bf a = as_v8bf(*reinterpret_cast<const v4u *>(sd + i * kDRow2 + c));
            const int plane = c / 120, within = c - 120 * plane;
            const int pc = 8 + within + 12 + 144 * (plane + 1);
            v4u bm, b0, bp;
            x_shifts(xrow + pc + 12 * ky + 144 * kz, bm, b0, bp);
            acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, as_v8bf(bm), acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, as_v8bf(b0), acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, as_v8bf(bp), acc[2], 0, 0, 0);
            if (wave < 3) {
                x_shifts(xrow + pc + 12 + 144, bm, b0, bp);
                acc[3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, as_v8bf(wave == 0 ? bm : (wave == 1 ? b0 : bp)),
                                                                 acc[3], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    float *out = partials + int64_t(blockIdx.x) * (kWPack + kC);
    // lane: column ci = i, rows co = 4g .. 4g + 3
    for (int j = 0; j < 4; ++j) {
        const int t = j < 3 ? 3 * wave + j : 24 + wave;
        if (j < 3 || wave < 3)
            for (int r = 0; r < 4; ++r) out[(t * kC + 4 * g + r) * kC + i] = acc[j][r];
    }
    sb[tid] = bsum;
    __syncthreads();
    if (tid < kC) {
        float sum = 0.f;
        for (int k = 0; k < 32; ++k) sum += sb[k * 16 + tid];
        out[kWPack + tid] = sum;
    }
}

static int pack_all(hipStream_t st, const float *params, uint16_t *wp)
{
    hipLaunchKernelGGL(k_pack, dim3(grid1(kWPack)), dim3(256), 0, st, params + kW1, 16, 2, 0, wp);
    hipLaunchKernelGGL(k_pack, dim3(grid1(kWPack)), dim3(256), 0, st, params + kW2, 16, 16, 0, wp + kWPack);
    hipLaunchKernelGGL(k_pack, dim3(grid1(kWPack)), dim3(256), 0, st, params + kW3, 1, 16, 0, wp + 2 * kWPack);
    hipLaunchKernelGGL(k_pack, dim3(grid1(kWPack)), dim3(256), 0, st, params + kW1, 16, 2, 1, wp + 3 * kWPack);
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
    hipLaunchKernelGGL(k_conv, dim3(unsigned(n)), dim3(256), 0, st, x0, n, wp, wp + 3 * kWPack, params + kB1, 1,
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
    if ((rc = pack_all(st, params, ws.wpack))) return rc;
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
                                   size_t(4) * kWPack * 2 + 4096;
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
    int dev = 0, cus = 0;
    DN_HIP(hipGetDevice(&dev));
    DN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned grid2 = unsigned(std::min<int64_t>(n, int64_t(2) * std::max(cus, 1)));
    // weights, forward with the layer inputs kept
    hipLaunchKernelGGL(k_pack_train, dim3(grid1(kLaneW + kL2M * 64 * 8)), dim3(256), 0, st, params, ws.lanew,
                       ws.lanef);
    hipLaunchKernelGGL(k_net_fwd<true>, dim3(grid2), dim3(256), 0, st, (const int32_t *)nullptr,
                       (const uint32_t *)nullptr, tiles, (const uint8_t *)nullptr, n, 0, 0, ws.lanew, params,
                       int64_t(0), ws.rc, ws.x1cf, ws.h1cf, ws.h2cf, ws.gates);
    DN_HIP(hipGetLastError());
    // loss and its gradient on the centre
    double *lsum = ws.misc;   // [0] loss, [1] 1 / N (written by k_grad_final)
    hipLaunchKernelGGL(k_loss_train, dim3(unsigned(n)), dim3(512), 0, st, tiles, ws.rc, targets, mask, n, int(kind),
                       ws.d3, ws.d3cf, ws.tl, ws.tc);
    DN_HIP(hipGetLastError());
    // input gradients of layers 3 and 2
    hipLaunchKernelGGL(k_net_bwd, dim3(grid2), dim3(256), 0, st, ws.d3, ws.gates, n, ws.lanef, params, ws.d2cf,
                       ws.d1cf);
    DN_HIP(hipGetLastError());
    // weight gradients, one partial per workgroup and layer, summed in a fixed order
    const unsigned gw = unsigned(ws.nparts);
    const size_t lp = size_t(ws.nparts) * (kWPack + kC);
    hipLaunchKernelGGL(k_wgrad13, dim3(2 * gw), dim3(256), 0, st, ws.x1cf, ws.d1cf, ws.h2cf, ws.d3cf, n, ws.parts,
                       ws.parts + 2 * lp, int(gw));
    hipLaunchKernelGGL((k_wgrad_mfma<16, 16>), dim3(gw), dim3(512), 0, st, ws.h1cf, ws.d2cf, n, ws.parts + lp);
    hipLaunchKernelGGL(k_grad_final, dim3((3 * (kWPack + kC) + kFinalEntries - 1) / kFinalEntries), dim3(256), 0, st,
                       ws.parts, ws.nparts, ws.tl, ws.tc, n, lsum, grad);
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
        hipLaunchKernelGGL(k_net_fwd<false>, dim3(grid), dim3(256), 0, st, v->nbr, vp, v->f, v->emask, v->nb,
                           mode == DN_WARM_DUAL ? a : 0, int(mode), lanew, params, ps,
                           mode == DN_WARM_DUAL ? p0 : u0, (uint16_t *)nullptr, (uint16_t *)nullptr,
                           (uint16_t *)nullptr, (uint16_t *)nullptr);
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
