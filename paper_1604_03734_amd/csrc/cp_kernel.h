// Device code of one fused Chambolle-Pock iteration on one 8^3 block,
// shared by the per-iteration kernel and the persistent batched kernel.
// Section III-B/C of the paper: Eq. (3) gradient, Eq. (4) divergence,
// Eqs. (7)-(9) updates.
#pragma once

#include "dn_internal.h"

namespace dn {

// ---------------------------------------------------------- storage types
// State storage: float, IEEE half or bfloat16 (16-bit kept as raw bits).
// sr(x, r) rounds stochastically with the 16 random bits r: the magnitude
// goes up one step with probability equal to the fraction of the step it
// has past the lower neighbour (adding random bits below the kept mantissa,
// then truncating), so rounding errors have mean zero and increments far
// below one step still accumulate.  Rounding to nearest (or toward zero)
// stalls the iteration once its increments drop below half a step.
struct SF32 {
    using T = float;
    static constexpr bool kLow = false;
    static __device__ __forceinline__ float ld(float v) { return v; }
    static __device__ __forceinline__ float rn(float x) { return x; }
    static __device__ __forceinline__ float rz(float x) { return x; }
    static __device__ __forceinline__ float sr(float x, uint32_t) { return x; }
};
struct SF16 {
    using T = uint16_t;
    static constexpr bool kLow = true;
    static __device__ __forceinline__ float ld(uint16_t v) { return float(__builtin_bit_cast(_Float16, v)); }
    static __device__ __forceinline__ uint16_t rn(float x) { return __builtin_bit_cast(uint16_t, _Float16(x)); }
    static __device__ __forceinline__ uint16_t rz(float x)
    {
        auto h2 = __builtin_amdgcn_cvt_pkrtz(x, 0.0f);
        return __builtin_bit_cast(uint16_t, h2[0]);
    }
    // 13 float mantissa bits fall away for a normal half (exact stochastic
    // rounding there; below 2^-14 the step is finer than the noise)
    static __device__ __forceinline__ uint16_t sr(float x, uint32_t r)
    {
        return rz(__uint_as_float(__float_as_uint(x) + (r & 0x1FFFu)));
    }
};
struct SBF16 {
    using T = uint16_t;
    static constexpr bool kLow = true;
    static __device__ __forceinline__ float ld(uint16_t v) { return __uint_as_float(uint32_t(v) << 16); }
    static __device__ __forceinline__ uint16_t rn(float x)
    {
        uint32_t u = __float_as_uint(x);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return uint16_t(u >> 16);
    }
    static __device__ __forceinline__ uint16_t rz(float x) { return uint16_t(__float_as_uint(x) >> 16); }
    static __device__ __forceinline__ uint16_t sr(float x, uint32_t r)
    {
        return uint16_t((__float_as_uint(x) + (r & 0xFFFFu)) >> 16);
    }
};

// Streaming accesses.  A block's f, w and u are read by that block alone
// and every store of the iteration is read back only in the next one (from
// HBM, the volume being far larger than the caches), whereas ubar, p and
// the edge masks are also read by the neighbours as their halo.  Loading
// the former and storing everything as non-temporal leaves the L2 for the
// lines the neighbouring blocks will read.
#ifndef DN_CP_NT
#define DN_CP_NT 1
#endif
template <class T> __device__ __forceinline__ T ld_stream(const T *p)
{
#if DN_CP_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}
template <class T> __device__ __forceinline__ void st_stream(T *p, T v)
{
#if DN_CP_NT
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// Counter-based random bits of one voxel and iteration: an integer hash
// (xor-shift / multiply rounds) of the global voxel index, a stream number
// and the iteration seed.  Deterministic, so a run is reproducible and a
// voxel's stored value does not depend on which workgroup wrote it.
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ uint32_t voxel_bits(int64_t gi, uint32_t stream, uint32_t seed)
{
    return mix32(uint32_t(gi) * 3u + stream + mix32(seed ^ uint32_t(uint64_t(gi) >> 32)));
}

template <class S> struct CPArgs {
    int64_t nb;                 // blocks
    int64_t pstride;            // elements between p planes
    const int32_t *nbr;         // [nb][27]
    const uint8_t *emask;       // [nb][512]
    const int32_t *order;       // processing order or nullptr (pool order)
    int32_t xcd;                // 1: XCD-chunked workgroup -> block map
    const float *f, *w;
    typename S::T *u;           // in place
    const typename S::T *ubar_in;
    typename S::T *ubar_out;
    const typename S::T *p_in;  // 3 planes
    typename S::T *p_out;
    float *u32, *ubar32, *p32;  // FP32 copies written by a refinement sweep
    float sigma, tau, lambda, theta;
    int32_t l1;                 // data term lambda w |u - f| (with u in [-1, 1]) instead of (lambda/2) w (u - f)^2
    uint32_t seed;              // 16-bit storage: this iteration's seed of the stochastic rounding
};

__device__ __forceinline__ int i10(int x, int y, int z) { return ((z + 1) * 10 + (y + 1)) * 10 + (x + 1); }
__device__ __forceinline__ int i9(int x, int y, int z) { return ((z + 1) * 9 + (y + 1)) * 9 + (x + 1); }

// Global index of voxel (hx, hy, hz) relative to block b, hx.. in [-1, 8],
// or -1 if it lies in an unallocated block.
__device__ __forceinline__ int64_t halo_index(const int32_t *nb27, int hx, int hy, int hz)
{
    int dx = hx < 0 ? -1 : (hx > 7 ? 1 : 0);
    int dy = hy < 0 ? -1 : (hy > 7 ? 1 : 0);
    int dz = hz < 0 ? -1 : (hz > 7 ? 1 : 0);
    int32_t id = nb27[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
    if (id < 0) return -1;
    return int64_t(id) * kBlockVox + ((hx - 8 * dx) + 8 * (hy - 8 * dy) + 64 * (hz - 8 * dz));
}

// Position of the t-th ubar halo voxel (t < 432): the six faces (+x, +y,
// +z, -x, -y, -z; 64 each) then the six (-a, +b) edges (8 each).
__device__ __forceinline__ void halo_pos(int t, int &x, int &y, int &z)
{
    if (t < 384) {
        int f = t >> 6, i = t & 63, a = i & 7, b = i >> 3;
        switch (f) {
        case 0: x = 8; y = a; z = b; break;
        case 1: x = a; y = 8; z = b; break;
        case 2: x = a; y = b; z = 8; break;
        case 3: x = -1; y = a; z = b; break;
        case 4: x = a; y = -1; z = b; break;
        default: x = a; y = b; z = -1; break;
        }
    } else {
        int e = (t - 384) >> 3, j = (t - 384) & 7;
        switch (e) {
        case 0: x = -1; y = 8; z = j; break;
        case 1: x = -1; y = j; z = 8; break;
        case 2: x = 8; y = -1; z = j; break;
        case 3: x = j; y = -1; z = 8; break;
        case 4: x = 8; y = j; z = -1; break;
        default: x = j; y = 8; z = -1; break;
        }
    }
}

// -1 face voxel e < 192: face 0 (-x), 1 (-y), 2 (-z)
__device__ __forceinline__ void face_pos(int t, int &x, int &y, int &z)
{
    int f = t >> 6, i = t & 63, a = i & 7, b = i >> 3;
    if (f == 0) { x = -1; y = a; z = b; }
    else if (f == 1) { x = a; y = -1; z = b; }
    else { x = a; y = b; z = -1; }
}

struct CPShared {
    float u[1000];       // ubar tile with a one-voxel halo, index i10
    float p[3][729];     // new dual on the block and its -1 faces, index i9
    uint8_t m[729];      // edge masks on the block and its -1 faces
};

__device__ __forceinline__ void project(float &a, float &b, float &c)
{
    float n = sqrtf((a * a + b * b) + c * c);
    if (n > 1.0f) { a = a / n; b = b / n; c = c / n; }
}

// Per-thread registers of one block's iteration: the thread's own voxels
// (VPT = 512 / NT of them), its share of the ubar halo (432 voxels: six
// faces and the six (-a, +b) edges) and its share of the 192 voxels of the
// -1 faces (their edge masks and the three dual components).
template <int NT> struct CPRegs {
    static constexpr int VPT = kBlockVox / NT;
    static constexpr int HPT = (432 + NT - 1) / NT;
    static constexpr int FPT = (192 + NT - 1) / NT;
    float ub[VPT], p0[VPT], p1[VPT], p2[VPT], uo[VPT], fv[VPT], wv[VPT];
    uint8_t m[VPT];
    float hu[HPT];
    float h0[FPT], h1[FPT], h2[FPT];
    uint8_t hm[FPT];
};

// Global loads of one block's iteration (issued; used by cp_compute).
template <class S, int NT>
__device__ __forceinline__ void cp_load(const CPArgs<S> &A, int64_t b, CPRegs<NT> &R, int t)
{
    constexpr int VPT = CPRegs<NT>::VPT, HPT = CPRegs<NT>::HPT;
    const int64_t g0i = b * kBlockVox;
    const int32_t *nb27 = A.nbr + b * kNbr;
    const int64_t ps = A.pstride;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int64_t gi = g0i + t + k * NT;
        R.ub[k] = S::ld(A.ubar_in[gi]);
        R.m[k] = A.emask[gi];
        R.p0[k] = S::ld(A.p_in[gi]); R.p1[k] = S::ld(A.p_in[gi + ps]); R.p2[k] = S::ld(A.p_in[gi + 2 * ps]);
        R.uo[k] = S::ld(ld_stream(A.u + gi));
        R.fv[k] = ld_stream(A.f + gi); R.wv[k] = ld_stream(A.w + gi);
    }
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
        const int h = t + k * NT;
        R.hu[k] = 0.0f;
        if (h < 432) {
            int hx, hy, hz;
            halo_pos(h, hx, hy, hz);
            int64_t j = halo_index(nb27, hx, hy, hz);
            if (j >= 0) R.hu[k] = S::ld(A.ubar_in[j]);
        }
    }
#pragma unroll
    for (int k = 0; k < CPRegs<NT>::FPT; ++k) {
        const int e = t + k * NT;
        R.h0[k] = R.h1[k] = R.h2[k] = 0.f;
        R.hm[k] = 0;
        if (e < 192) {
            int fx, fy, fz;
            face_pos(e, fx, fy, fz);
            int64_t j = halo_index(nb27, fx, fy, fz);
            if (j >= 0) {
                R.hm[k] = A.emask[j];
                R.h0[k] = S::ld(A.p_in[j]); R.h1[k] = S::ld(A.p_in[j + ps]); R.h2[k] = S::ld(A.p_in[j + 2 * ps]);
            }
        }
    }
}

// The iteration of one block from its loaded registers (NT threads: 512 =
// one voxel per thread; 256 = two voxels per thread, z layers l and l + 4).
template <class S, bool kRefine, int NT>
__device__ __forceinline__ void cp_compute(const CPArgs<S> &A, int64_t b, const CPRegs<NT> &R, CPShared &sh,
                                           int t)
{
    constexpr int VPT = CPRegs<NT>::VPT, HPT = CPRegs<NT>::HPT;
    const int64_t g0i = b * kBlockVox;
    const int64_t ps = A.pstride;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int v = t + k * NT, lx = v & 7, ly = (v >> 3) & 7, lz = v >> 6;
        sh.u[i10(lx, ly, lz)] = R.ub[k];
        sh.m[i9(lx, ly, lz)] = R.m[k];
    }
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
        const int h = t + k * NT;
        if (h < 432) {
            int hx, hy, hz;
            halo_pos(h, hx, hy, hz);
            sh.u[i10(hx, hy, hz)] = R.hu[k];
        }
    }
#pragma unroll
    for (int k = 0; k < CPRegs<NT>::FPT; ++k) {
        const int e = t + k * NT;
        if (e < 192) {
            int fx, fy, fz;
            face_pos(e, fx, fy, fz);
            sh.m[i9(fx, fy, fz)] = R.hm[k];
        }
    }
    __syncthreads();

    // dual ascent and projection on the block (Eq. 7)
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int v = t + k * NT, lx = v & 7, ly = (v >> 3) & 7, lz = v >> 6;
        const int64_t gi = g0i + v;
        const uint8_t m = R.m[k];
        float g0 = (m & 2) ? sh.u[i10(lx + 1, ly, lz)] - R.ub[k] : 0.0f;
        float g1 = (m & 4) ? sh.u[i10(lx, ly + 1, lz)] - R.ub[k] : 0.0f;
        float g2 = (m & 8) ? sh.u[i10(lx, ly, lz + 1)] - R.ub[k] : 0.0f;
        float a0 = R.p0[k] + A.sigma * g0, a1 = R.p1[k] + A.sigma * g1, a2 = R.p2[k] + A.sigma * g2;
        project(a0, a1, a2);
        const int q = i9(lx, ly, lz);
        sh.p[0][q] = a0; sh.p[1][q] = a1; sh.p[2][q] = a2;
        if constexpr (S::kLow) {
            // stochastic rounding; where it would leave the unit ball, toward zero
            const uint32_t r0 = voxel_bits(gi, 0, A.seed), r1 = voxel_bits(gi, 1, A.seed);
            typename S::T s0 = S::sr(a0, r0), s1 = S::sr(a1, r0 >> 16), s2 = S::sr(a2, r1);
            const float b0 = S::ld(s0), b1 = S::ld(s1), b2 = S::ld(s2);
            if ((b0 * b0 + b1 * b1) + b2 * b2 > 1.0f) { s0 = S::rz(a0); s1 = S::rz(a1); s2 = S::rz(a2); }
            st_stream(A.p_out + gi, s0); st_stream(A.p_out + gi + ps, s1); st_stream(A.p_out + gi + 2 * ps, s2);
        } else {
            st_stream(A.p_out + gi, a0); st_stream(A.p_out + gi + ps, a1); st_stream(A.p_out + gi + 2 * ps, a2);
        }
        if (kRefine) { A.p32[gi] = a0; A.p32[gi + ps] = a1; A.p32[gi + 2 * ps] = a2; }
    }
    // ... and on the -1 faces, which the divergence needs
#pragma unroll
    for (int k = 0; k < CPRegs<NT>::FPT; ++k) {
        const int e = t + k * NT;
        if (e < 192) {
            int fx, fy, fz;
            face_pos(e, fx, fy, fz);
            const uint8_t hm = R.hm[k];
            float uh = sh.u[i10(fx, fy, fz)];
            float g0 = (hm & 2) ? sh.u[i10(fx + 1, fy, fz)] - uh : 0.0f;
            float g1 = (hm & 4) ? sh.u[i10(fx, fy + 1, fz)] - uh : 0.0f;
            float g2 = (hm & 8) ? sh.u[i10(fx, fy, fz + 1)] - uh : 0.0f;
            float h0 = R.h0[k] + A.sigma * g0, h1 = R.h1[k] + A.sigma * g1, h2 = R.h2[k] + A.sigma * g2;
            project(h0, h1, h2);
            const int q = i9(fx, fy, fz);
            sh.p[0][q] = h0; sh.p[1][q] = h1; sh.p[2][q] = h2;
        }
    }
    __syncthreads();

    // primal proximal step (Eq. 8) and relaxation (Eq. 9)
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int v = t + k * NT, lx = v & 7, ly = (v >> 3) & 7, lz = v >> 6;
        const int64_t gi = g0i + v;
        const uint8_t m = R.m[k];
        float un = R.uo[k];
        if (m & 1) {
            const int q = i9(lx, ly, lz);
            const int qx = i9(lx - 1, ly, lz), qy = i9(lx, ly - 1, lz), qz = i9(lx, ly, lz - 1);
            float dv = 0.0f;
            dv += ((m & 2) ? sh.p[0][q] : 0.0f) - ((sh.m[qx] & 2) ? sh.p[0][qx] : 0.0f);
            dv += ((m & 4) ? sh.p[1][q] : 0.0f) - ((sh.m[qy] & 4) ? sh.p[1][qy] : 0.0f);
            dv += ((m & 8) ? sh.p[2][q] : 0.0f) - ((sh.m[qz] & 8) ? sh.p[2][qz] : 0.0f);
            float ut = R.uo[k] + A.tau * dv;
            float tlw = A.tau * A.lambda * R.wv[k];
            if (A.l1) {
                // soft threshold of u~ - f by tau lambda w, then the [-1, 1] box
                float r = ut - R.fv[k];
                r = r > tlw ? r - tlw : (r < -tlw ? r + tlw : 0.0f);
                un = fminf(fmaxf(R.fv[k] + r, -1.0f), 1.0f);
            } else {
                un = (ut + tlw * R.fv[k]) / (1.0f + tlw);
            }
        }
        float ubn = un + A.theta * (un - R.uo[k]);
        if constexpr (S::kLow) {
            const uint32_t r2 = voxel_bits(gi, 2, A.seed);
            st_stream(A.u + gi, S::sr(un, r2));
            st_stream(A.ubar_out + gi, S::sr(ubn, r2 >> 16));
        } else {
            st_stream(A.u + gi, un);
            st_stream(A.ubar_out + gi, ubn);
        }
        if (kRefine) { A.u32[gi] = un; A.ubar32[gi] = ubn; }
    }
}

// One fused Chambolle-Pock iteration on block b by NT threads.  t is the
// thread index (a loop that runs many blocks passes it through an opaque
// copy so that the per-thread index arithmetic is redone per block instead
// of being kept live across the loop).
template <class S, bool kRefine, int NT = 512>
__device__ __forceinline__ void cp_block(const CPArgs<S> &A, int64_t b, CPShared &sh, int t)
{
    CPRegs<NT> R;
    cp_load<S, NT>(A, b, R, t);
    cp_compute<S, kRefine, NT>(A, b, R, sh, t);
}

// threadIdx.x that the compiler cannot hoist out of an enclosing loop
__device__ __forceinline__ int opaque_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Workgroup -> block mapping.  Consecutive workgroups go round-robin to the
// 8 XCDs; giving XCD x the x-th contiguous chunk of the (Morton) order keeps
// spatial neighbours, whose faces are each other's halos, in one L2.
__device__ __forceinline__ int64_t xcd_slot(int64_t wg, int64_t n)
{
    int64_t per = (n + 7) / 8;
    return (wg % 8) * per + wg / 8;
}

__device__ __forceinline__ int64_t block_slot(int64_t wg, int64_t n, int xcd)
{
    return xcd ? xcd_slot(wg, n) : wg;
}

}  // namespace dn
