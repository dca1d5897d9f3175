// Many sub-maps in one HIP graph (gfx950).
//
// All (sub-map, block) work items of every volume run in one kernel that
// loops over the iterations itself; a grid-wide barrier separates one
// iteration from the next (the fused iteration reads its neighbours' ubar
// and p of the previous iteration).  The other candidate launches one
// iteration of every sub-map per kernel, the launch boundary ordering the
// iterations.  Either is captured in a HIP graph together with the reset
// of the barrier state and replayed.  Kernel, grid size and the
// item-to-workgroup mapping are picked by timing short trial runs
// (autotuner), cached per problem size.
#include <cstring>
#include <cstdlib>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "cp_kernel.h"
#include "dn_internal.h"

namespace dn {

struct VolDesc {
    const int32_t *nbr;
    const uint8_t *emask;
    const float *f, *w;
    float *u;
    float *ubar[2];
    float *p[2];
    int64_t pstride;
    int32_t cur;
    int32_t pad;
};

struct BatchArgs {
    const VolDesc *vols;
    const int2 *items;        // (volume, block) in processing order
    int64_t n_items;
    int32_t iters;
    int32_t xcd_chunks;       // 1: each XCD works on one contiguous item chunk
    float sigma, tau, lambda, theta;
    double gamma;             // > 0: accelerated schedule from (tau, sigma)
    double tau0, sigma0;      // schedule state at the start of the launch
    unsigned *bar;            // barrier state, kBarWords words (layout below)
    int32_t *err;             // set when a barrier wait exceeds its bound
    long long spin_limit;
    int32_t l1;               // L1 data term
};

// Barrier state: one 256-byte slot per word that is written concurrently,
// so arrivals and polls of different groups never share a cache line.
// slot 0: arrivals of group leaders, slot 1: generation, slot 2: error flag,
// slots 3 .. 3+kBarMaxGroups-1: arrivals per group, then one release flag
// per group, then the item counters of the eight XCD chunks.  All zeroed
// before every launch.
constexpr int kBarSlot = 64;
constexpr int kBarGroup = 32;
constexpr int kBarMaxGroups = 256;
constexpr int kBarCtr = (3 + 2 * kBarMaxGroups) * kBarSlot;   // then 8 item counters, one slot each
constexpr int kBarWords = kBarCtr + 8 * kBarSlot;
constexpr int kBarMaxGrid = kBarGroup * kBarMaxGroups;

__global__ void k_batch_reset(unsigned *bar)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kBarWords; i += gridDim.x * blockDim.x)
        bar[i] = 0u;
}

// Bounded wait until *word >= target; false (and the error flag raised) if
// the bound is exceeded or another workgroup already raised it.  The polls
// are relaxed: an acquiring load invalidates the L2 of its XCD on every
// poll, which would evict the data of the workgroups still computing; the
// caller places one acquire fence after the wait instead.
__device__ __forceinline__ bool wait_at_least(const BatchArgs &a, unsigned *word, unsigned target)
{
    long long spins = 0;
    while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        __builtin_amdgcn_s_sleep(2);
        if (++spins > a.spin_limit) {
            __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// Two-level grid barrier number `target` (1, 2, ... within a launch).
// Workgroups arrive in groups of kBarGroup; the last arrival of a group
// (its leader) arrives at the top counter and waits for the generation,
// the last leader publishes it; each leader then releases its group
// through the group's own flag.  Every poll and every atomic of one group
// touches only that group's lines.  Ordering uses explicit agent-scope
// fences around relaxed atomics: a release fence before each arrival, an
// acquire fence after each observed arrival or release, so every
// workgroup's writes of this iteration happen before every read of the
// next.  Every wait is bounded: past spin_limit polls the error flag is
// raised and every waiter returns, so the grid always drains.
__device__ __forceinline__ void grid_barrier(const BatchArgs &a, unsigned nwg, unsigned target)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned grp = blockIdx.x / kBarGroup;
        const unsigned ngrp = (nwg + kBarGroup - 1) / kBarGroup;
        const unsigned gsize = min(unsigned(kBarGroup), nwg - grp * kBarGroup);
        unsigned *cnt = a.bar + (3 + grp) * kBarSlot;
        unsigned *flag = a.bar + (3 + kBarMaxGroups + grp) * kBarSlot;
        unsigned *top = a.bar;
        unsigned *gen = a.bar + kBarSlot;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned prev = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gsize - 1u) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned p2 = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (p2 == ngrp - 1u) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(gen, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                (void)wait_at_least(a, gen, target);
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            }
            __hip_atomic_store(flag, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            (void)wait_at_least(a, flag, target);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// The item of a workgroup is the same for all its lanes: read it through
// readfirstlane so the volume's pointers live in scalar registers.
__device__ __forceinline__ int2 load_item(const int2 *__restrict__ items, int64_t i)
{
    const int2 raw = items[i];
    return make_int2(__builtin_amdgcn_readfirstlane(raw.x), __builtin_amdgcn_readfirstlane(raw.y));
}

// A pointer the whole wave shares, moved to scalar registers.  The volume
// buffers are global memory; rebuilding the pointer in the global address
// space lets the compiler address them with global instructions (through
// a generic pointer it would emit flat ones, which count against the LDS
// wait counter too, so every LDS wait would also wait for the loads).
template <class T> __device__ __forceinline__ T *uni(T *p)
{
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    typedef __attribute__((address_space(1))) T GT;
    return (T *)reinterpret_cast<GT *>((uint64_t(hi) << 32) | lo);
}

__device__ __forceinline__ void item_args(const BatchArgs &a, const VolDesc *__restrict__ vols, int2 item, int it,
                                          float sigma, float tau, float theta, CPArgs<SF32> &A)
{
    const VolDesc &d = vols[item.x];
    const int c = (__builtin_amdgcn_readfirstlane(d.cur) + it) & 1;
    const int64_t ps = int64_t(__builtin_amdgcn_readfirstlane(uint32_t(d.pstride))) |
                       (int64_t(__builtin_amdgcn_readfirstlane(uint32_t(uint64_t(d.pstride) >> 32))) << 32);
    A.nb = 0; A.pstride = ps; A.nbr = uni(d.nbr); A.emask = uni(d.emask); A.order = nullptr; A.xcd = 0;
    A.f = uni(d.f); A.w = uni(d.w); A.u = uni(d.u);
    A.ubar_in = uni(d.ubar[c]); A.ubar_out = uni(d.ubar[1 - c]);
    A.p_in = uni(d.p[c]); A.p_out = uni(d.p[1 - c]); A.u32 = nullptr; A.ubar32 = nullptr; A.p32 = nullptr;
    A.sigma = sigma; A.tau = tau; A.lambda = a.lambda; A.theta = theta;
    A.l1 = a.l1;
    A.seed = 0u;
}

// All iterations of all sub-maps.  Without kPrefetch the workgroups take
// the items of an iteration from a shared counter (per XCD chunk); with
// kPrefetch each walks a fixed stride of them and issues the global loads
// of the next item before computing the current one (two register sets, so
// loads stay in flight while it works).  A grid barrier closes every
// iteration.
template <int NT, bool kPrefetch>
__device__ __forceinline__ void k_cp_persistent_body(const BatchArgs &a, const VolDesc *__restrict__ vols,
                                                     const int2 *__restrict__ items)
{
    __shared__ CPShared sh;
    __shared__ int s_stop;
    __shared__ unsigned s_next;
    const unsigned nwg = gridDim.x;
    const int64_t G = nwg;
    double acc_tau = a.tau0, acc_sigma = a.sigma0;
    for (int it = 0; it < a.iters; ++it) {
        float sigma = a.sigma, tau = a.tau, theta = a.theta;
        if (a.gamma > 0.0) {
            const double th = 1.0 / sqrt(1.0 + 2.0 * a.gamma * acc_tau);
            tau = float(acc_tau);
            sigma = float(acc_sigma);
            theta = float(th);
            acc_tau = th * acc_tau;
            acc_sigma = acc_sigma / th;
        }
        int64_t i, hi, stride, lo = 0, cx = 0;
        if (a.xcd_chunks && G >= 8) {
            // workgroup g runs on XCD g % 8; XCD x owns items [x*chunk, (x+1)*chunk)
            // and has exactly (G - x + 7) / 8 workgroups to stride over them
            const int64_t x = blockIdx.x % 8, lane = blockIdx.x / 8;
            const int64_t chunk = (a.n_items + 7) / 8;
            lo = x * chunk;
            hi = min(a.n_items, lo + chunk);
            stride = (G - x + 7) / 8;
            i = lo + lane;
            cx = x;
        } else {
            i = blockIdx.x;
            hi = a.n_items;
            stride = G;
        }
        if constexpr (!kPrefetch) {
            // One block after the other (the other workgroups on the CU
            // overlap), each taken in order from the items [lo, hi) through
            // the chunk's counter, so that the items in flight stay one
            // contiguous window however unevenly the workgroups progress.
            // The next index is taken while the current block is processed.
            // Every workgroup of the chunk ends an iteration with exactly one
            // index past the end, so the counter advances by len + stride per
            // iteration and the index is its value less that base (modulo
            // 2^32, which keeps differences exact).
            unsigned *ctr = a.bar + kBarCtr + cx * kBarSlot;
            const unsigned len = unsigned(hi > lo ? hi - lo : 0);
            const unsigned base = unsigned(it) * (len + unsigned(stride));
            if (threadIdx.x == 0)
                s_next = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - base;
            __syncthreads();
            unsigned rel = s_next;
            while (rel < len) {
                unsigned nraw = 0;
                __syncthreads();   // every thread has read s_next
                if (threadIdx.x == 0)
                    nraw = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int2 bi = load_item(items, lo + rel);
                CPArgs<SF32> A;
                item_args(a, vols, bi, it, sigma, tau, theta, A);
                cp_block<SF32, false, NT>(A, bi.y, sh, opaque_tid());
                if (threadIdx.x == 0) s_next = nraw - base;
                __syncthreads();
                rel = s_next;
            }
        } else {
        CPRegs<NT> R0, R1;
        CPArgs<SF32> A0, A1;
        int2 b0 = make_int2(0, 0), b1 = make_int2(0, 0);
        if (i < hi) {
            b0 = load_item(items, i);
            item_args(a, vols, b0, it, sigma, tau, theta, A0);
            cp_load<SF32, NT>(A0, b0.y, R0, opaque_tid());
        }
        while (i < hi) {
            int64_t nx = i + stride;
            if (nx < hi) {
                b1 = load_item(items, nx);
                item_args(a, vols, b1, it, sigma, tau, theta, A1);
                cp_load<SF32, NT>(A1, b1.y, R1, opaque_tid());
            }
            cp_compute<SF32, false, NT>(A0, b0.y, R0, sh, opaque_tid());
            __syncthreads();
            i = nx;
            if (i >= hi) break;
            nx = i + stride;
            if (nx < hi) {
                b0 = load_item(items, nx);
                item_args(a, vols, b0, it, sigma, tau, theta, A0);
                cp_load<SF32, NT>(A0, b0.y, R0, opaque_tid());
            }
            cp_compute<SF32, false, NT>(A1, b1.y, R1, sh, opaque_tid());
            __syncthreads();
            i = nx;
        }
        }
        grid_barrier(a, nwg, unsigned(it + 1));
        if (threadIdx.x == 0)
            s_stop = __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        if (s_stop) return;
    }
}

// The descriptors and the item list (read-only during the launch) are also
// passed as restrict-qualified kernel arguments: no store of the loop can
// then alias them, so the compiler reads them with scalar loads, which
// shortens the chain of dependent loads in front of each block.
template <int NT, bool kPrefetch>
__global__ __launch_bounds__(NT) void k_cp_persistent(BatchArgs a, const VolDesc *__restrict__ vols,
                                                     const int2 *__restrict__ items)
{
    k_cp_persistent_body<NT, kPrefetch>(a, vols, items);
}

// The lean form: no prefetch, registers capped for 8 waves per SIMD.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_cp_persistent_lean(
    BatchArgs a, const VolDesc *__restrict__ vols, const int2 *__restrict__ items)
{
    k_cp_persistent_body<256, false>(a, vols, items);
}

// One iteration of every sub-map: one workgroup per item, the items
// mapped to workgroups in XCD chunks as in the single-map kernel (so the
// blocks in flight are a contiguous window of the item list per XCD, as
// hardware dispatch keeps them); no barrier, the next launch is the next
// iteration.
constexpr int kStepKernel = 1;   // variant code of this kernel in the tuner
__global__ __launch_bounds__(256) void k_cp_batch_step(BatchArgs a, const VolDesc *__restrict__ vols,
                                                       const int2 *__restrict__ items, int it, float sigma,
                                                       float tau, float theta)
{
    __shared__ CPShared sh;
    const int64_t slot = block_slot(blockIdx.x, a.n_items, a.xcd_chunks);
    if (slot >= a.n_items) return;
    const int2 bi = load_item(items, slot);
    CPArgs<SF32> A;
    item_args(a, vols, bi, it, sigma, tau, theta, A);
    cp_block<SF32, false, 256>(A, bi.y, sh, threadIdx.x);
}

__global__ void k_make_items(const int32_t *__restrict__ order, int64_t nb, int32_t vol, int2 *__restrict__ items)
{
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nb) items[i] = make_int2(vol, order ? order[i] : int32_t(i));
}

// Per-device batch context: the cached graph and the private stream it is
// captured on and replayed on (the device buffers are the caller's workspace).
struct BatchCtx {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // key of the captured graph
    const void *k_items = nullptr;
    int64_t k_n = -1;
    int k_iters = -1, k_grid = -1, k_xcd = -1, k_nt = -1, k_l1 = -1;
    float k_prm[4] = {0, 0, 0, 0};
    double k_acc[3] = {0, 0, 0};
    const void *vols_ptr = nullptr;
    const void *bar_ptr = nullptr;
    hipStream_t cap = nullptr;        // private stream for capture and replay
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
};
static std::map<int, BatchCtx> g_batch;     // by device
static std::mutex g_batch_mutex;             // held for a whole batched call

// (threads per workgroup, workgroups per CU, XCD-chunked items, pool order)
struct TuneChoice { int nt; int wg_per_cu; int xcd; int pool; };
static std::map<int64_t, TuneChoice> g_tuned;   // by (device, size bucket)

// The workspace of one batched call: volume descriptors, work items and
// the barrier state.
struct BatchWS {
    VolDesc *descs;
    int2 *items;
    unsigned *state;
};
static BatchWS carve_batch(Bump &b, int32_t n, int64_t total)
{
    BatchWS x;
    x.descs = b.take<VolDesc>(size_t(n));
    x.items = b.take<int2>(size_t(total > 0 ? total : 1));
    x.state = b.take<unsigned>(size_t(kBarWords));
    return x;
}

static int size_bucket(int64_t n)
{
    int b = 0;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

// variant: 256 / 512 = threads per workgroup with prefetch of the next
// block; 257 = 256 threads without prefetch (fewer registers, more
// workgroups per CU); kStepKernel = one launch per iteration (grid
// unused).  The step sizes of the accelerated schedule are formed as the
// persistent kernel forms them (double precision, the same operations).
static void launch_kernel(hipStream_t st, const BatchArgs &a, int grid, int nt)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(32), dim3(256), 0, st, a.bar);
    if (nt == kStepKernel) {
        const unsigned g = unsigned(((a.n_items + 7) / 8) * 8);
        double acc_tau = a.tau0, acc_sigma = a.sigma0;
        for (int it = 0; it < a.iters; ++it) {
            float sigma = a.sigma, tau = a.tau, theta = a.theta;
            if (a.gamma > 0.0) {
                const double th = 1.0 / std::sqrt(1.0 + 2.0 * a.gamma * acc_tau);
                tau = float(acc_tau);
                sigma = float(acc_sigma);
                theta = float(th);
                acc_tau = th * acc_tau;
                acc_sigma = acc_sigma / th;
            }
            hipLaunchKernelGGL(k_cp_batch_step, dim3(g), dim3(256), 0, st, a, a.vols, a.items, it, sigma, tau,
                               theta);
        }
    } else if (nt == 256)
        hipLaunchKernelGGL((k_cp_persistent<256, true>), dim3(grid), dim3(256), 0, st, a, a.vols, a.items);
    else if (nt == 257)
        hipLaunchKernelGGL(k_cp_persistent_lean, dim3(grid), dim3(256), 0, st, a, a.vols, a.items);
    else
        hipLaunchKernelGGL((k_cp_persistent<512, true>), dim3(grid), dim3(512), 0, st, a, a.vols, a.items);
}

static int launch_direct(hipStream_t st, const BatchArgs &a, int grid, int nt)
{
    launch_kernel(st, a, grid, nt);
    DN_HIP(hipGetLastError());
    return DN_OK;
}

// Capture (once per configuration) and replay on a private stream that is
// ordered after and before the caller's stream with events (the caller's
// stream may be the null stream, which cannot be captured).
static int launch_graph(BatchCtx &c, hipStream_t st, const BatchArgs &a, int grid, int nt)
{
    if (!c.cap) {
        DN_HIP(hipStreamCreateWithFlags(&c.cap, hipStreamNonBlocking));
        DN_HIP(hipEventCreateWithFlags(&c.ev_in, hipEventDisableTiming));
        DN_HIP(hipEventCreateWithFlags(&c.ev_out, hipEventDisableTiming));
    }
    bool same = c.exec && c.k_items == a.items && c.k_n == a.n_items && c.k_iters == a.iters && c.k_grid == grid &&
                c.k_nt == nt && c.k_l1 == a.l1 &&
                c.k_xcd == a.xcd_chunks && c.k_prm[0] == a.sigma && c.k_prm[1] == a.tau &&
                c.k_prm[2] == a.lambda && c.k_prm[3] == a.theta && c.vols_ptr == a.vols && c.bar_ptr == a.bar &&
                c.k_acc[0] == a.gamma && c.k_acc[1] == a.tau0 && c.k_acc[2] == a.sigma0;
    if (!same) {
        if (c.exec) { (void)hipGraphExecDestroy(c.exec); c.exec = nullptr; }
        if (c.graph) { (void)hipGraphDestroy(c.graph); c.graph = nullptr; }
        DN_HIP(hipStreamBeginCapture(c.cap, hipStreamCaptureModeThreadLocal));
        launch_kernel(c.cap, a, grid, nt);
        hipError_t le = hipGetLastError();
        hipError_t ce = hipStreamEndCapture(c.cap, &c.graph);
        if (le != hipSuccess || ce != hipSuccess) {
            set_error("graph capture failed: %s / %s", hipGetErrorString(le), hipGetErrorString(ce));
            return DN_E_DEVICE;
        }
        DN_HIP(hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0));
        c.k_items = a.items; c.k_n = a.n_items; c.k_iters = a.iters; c.k_grid = grid; c.k_xcd = a.xcd_chunks;
        c.k_nt = nt;
        c.k_l1 = a.l1;
        c.k_prm[0] = a.sigma; c.k_prm[1] = a.tau; c.k_prm[2] = a.lambda; c.k_prm[3] = a.theta;
        c.k_acc[0] = a.gamma; c.k_acc[1] = a.tau0; c.k_acc[2] = a.sigma0;
        c.vols_ptr = a.vols; c.bar_ptr = a.bar;
    }
    DN_HIP(hipEventRecord(c.ev_in, st));
    DN_HIP(hipStreamWaitEvent(c.cap, c.ev_in, 0));
    DN_HIP(hipGraphLaunch(c.exec, c.cap));
    DN_HIP(hipEventRecord(c.ev_out, c.cap));
    DN_HIP(hipStreamWaitEvent(st, c.ev_out, 0));
    return DN_OK;
}

static int check_err(dn_volume *v0, hipStream_t st, int32_t *err_dev)
{
    hipStream_t keep = v0->stream;
    v0->stream = st;
    int rc = read_back(v0, err_dev, 4);
    v0->stream = keep;
    if (rc) return rc;
    int32_t err = 0;
    memcpy(&err, v0->host_stage, 4);
    if (err != 0) {
        set_error("persistent kernel: a grid barrier wait exceeded its bound (workgroups not co-resident)");
        return DN_E_DEVICE;
    }
    return DN_OK;
}

}  // namespace dn

using namespace dn;

extern "C" size_t dn_regularize_batch_bytes(int32_t n, int64_t total_blocks)
{
    if (n <= 0 || total_blocks < 0) return 0;
    Bump b(nullptr, 0);
    carve_batch(b, n, total_blocks);
    return (b.off + 255) & ~size_t(255);
}

extern "C" int dn_regularize_batch(dn_volume *const *vols, int32_t n, const dn_reg_params *prm, void *workspace,
                                   size_t workspace_bytes, dn_reg_stats *out)
{
    DN_REQUIRE(vols && n > 0 && prm, "bad argument");
    DN_REQUIRE(workspace && (reinterpret_cast<uintptr_t>(workspace) & 255) == 0,
               "the workspace must be non-null and 256-byte aligned");
    DN_REQUIRE(prm->lambda > 0 && prm->tau > 0 && prm->sigma > 0 && prm->tau * prm->sigma * 12.0 <= 1.0 + 1e-9,
               "bad step sizes");
    DN_REQUIRE(prm->theta >= 0 && prm->theta <= 1 && prm->iters >= 0, "bad theta or iters");
    DN_REQUIRE(prm->storage == DN_F32, "the batched solver stores its state in FP32");
    DN_REQUIRE(prm->init == DN_INIT_ZERO || prm->init == DN_INIT_KEEP, "init must be ZERO or KEEP");
    DN_REQUIRE(prm->gamma >= 0 && std::isfinite(prm->gamma), "gamma must be >= 0");
    DN_REQUIRE(prm->data_term == DN_DATA_L2 || prm->data_term == DN_DATA_L1, "bad data_term");
    DN_REQUIRE(prm->data_term == DN_DATA_L2 || prm->gamma == 0.0,
               "the accelerated variant needs the uniformly convex (L2) data term");
    for (int i = 0; i < n; ++i) {
        DN_REQUIRE(vols[i], "null volume %d", i);
        DN_REQUIRE(vols[i]->device == vols[0]->device, "volumes on different devices");
    }
    dn_volume *v0 = vols[0];
    hipStream_t st = v0->stream;
    int rc;
    int64_t total = 0;
    for (int i = 0; i < n; ++i) total += vols[i]->nb;
    if (workspace_bytes < dn_regularize_batch_bytes(n, total)) {
        set_error("workspace of %zu bytes is short: %zu needed (dn_regularize_batch_bytes)", workspace_bytes,
                  dn_regularize_batch_bytes(n, total));
        return DN_E_CAPACITY;
    }
    std::lock_guard<std::mutex> lk(g_batch_mutex);
    BatchCtx &c = g_batch[v0->device];
    Bump bump(workspace, workspace_bytes);
    const BatchWS ws = carve_batch(bump, n, total);
    total = 0;
    for (int i = 0; i < n; ++i) {
        dn_volume *v = vols[i];
        // each volume's own work must be ordered before ours
        if (v->stream != st) DN_HIP(hipStreamSynchronize(v->stream));
        hipStream_t keep = v->stream;
        v->stream = st;
        rc = build_masks(v);
        if (!rc && prm->init == DN_INIT_ZERO) rc = zero_state(v);
        if (!rc && v->state_storage != DN_F32) v->state_storage = DN_F32;
        v->stream = keep;
        if (rc) return rc;
        total += v->nb;
    }
    std::vector<VolDesc> hd(n);
    for (int i = 0; i < n; ++i) {
        dn_volume *v = vols[i];
        VolDesc &d = hd[i];
        d.nbr = v->nbr; d.emask = v->emask; d.f = v->f; d.w = v->w; d.u = v->u;
        d.ubar[0] = v->ubar[0]; d.ubar[1] = v->ubar[1]; d.p[0] = v->p[0]; d.p[1] = v->p[1];
        d.pstride = v->cap_blocks * kBlockVox;
        d.cur = v->cur;
        d.pad = 0;
    }
    DN_HIP(hipMemcpyAsync(ws.descs, hd.data(), sizeof(VolDesc) * size_t(n), hipMemcpyHostToDevice, st));
    // work items (volume, block): volume after volume, blocks in Morton or pool order
    auto build_items = [&](int pool) -> int {
        int64_t ofs = 0;
        for (int i = 0; i < n; ++i) {
            dn_volume *v = vols[i];
            if (v->nb > 0) {
                hipLaunchKernelGGL(k_make_items, dim3(unsigned((v->nb + 255) / 256)), dim3(256), 0, st,
                                   pool ? (const int32_t *)nullptr : v->order, v->nb, i, ws.items + ofs);
                DN_HIP(hipGetLastError());
            }
            ofs += v->nb;
        }
        return DN_OK;
    };

    BatchArgs a;
    a.vols = ws.descs;
    a.items = ws.items;
    a.n_items = total;
    a.sigma = float(prm->sigma); a.tau = float(prm->tau); a.lambda = float(prm->lambda); a.theta = float(prm->theta);
    // the accelerated schedule of the batch lives in the first volume
    if (prm->init != DN_INIT_KEEP || v0->acc_tau <= 0.0) { v0->acc_tau = prm->tau; v0->acc_sigma = prm->sigma; }
    a.gamma = prm->gamma;
    a.tau0 = v0->acc_tau;
    a.sigma0 = v0->acc_sigma;
    a.bar = ws.state;
    a.err = reinterpret_cast<int32_t *>(ws.state + 2 * kBarSlot);
    a.spin_limit = 1LL << 22;
    a.xcd_chunks = 1;
    a.l1 = prm->data_term == DN_DATA_L1;

    // occupancy bound: every workgroup of the grid must be resident at once
    int dev_cu = 0, per_cu256 = 0, per_cu257 = 0, per_cu512 = 0;
    DN_HIP(hipDeviceGetAttribute(&dev_cu, hipDeviceAttributeMultiprocessorCount, v0->device));
    DN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu256, k_cp_persistent<256, true>, 256, 0));
    DN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu257, k_cp_persistent_lean, 256, 0));
    DN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu512, k_cp_persistent<512, true>, 512, 0));
    if (per_cu257 < 1) { set_error("persistent kernel does not fit on a compute unit"); return DN_E_DEVICE; }

    // DN_K_FUSED256: one launch of the fused kernel per iteration; other
    // explicit choices: the persistent kernel; both on the blocks in pool
    // order, XCD-chunked.  DN_K_AUTO: the tuned choice
    TuneChoice ch = TuneChoice{257, per_cu257, 1, 1};
    if (prm->kernel == DN_K_FUSED256) ch = TuneChoice{kStepKernel, 1, 1, 1};
    const int64_t key = (int64_t(v0->device) << 32) | size_bucket(total);
    auto it = g_tuned.find(key);
    const bool tuned = prm->kernel == DN_K_AUTO;
    if (tuned && it != g_tuned.end()) {
        ch = it->second;
    } else if (tuned && prm->init == DN_INIT_ZERO && total > 0 && prm->iters > 0) {
        // autotune: a few iterations of each candidate, from the zero state
        hipEvent_t e0, e1;
        DN_HIP(hipEventCreate(&e0));
        DN_HIP(hipEventCreate(&e1));
        float best = 1e30f;
        const int trial = std::min(prm->iters, 6);
        for (int pool = 0; pool <= 1; ++pool) {
            if ((rc = build_items(pool))) return rc;
            for (int nt : {257, 256, 512, kStepKernel}) {
                const int pc = nt == kStepKernel ? 1 : (nt == 256 ? per_cu256 : (nt == 257 ? per_cu257 : per_cu512));
                if (pc < 1) continue;
                std::vector<int> wpcs = {pc};
                if ((pc + 1) / 2 != pc) wpcs.push_back((pc + 1) / 2);
                for (int wpc : wpcs) {
                    for (int xcd = 0; xcd <= 1; ++xcd) {
                        BatchArgs t = a;
                        t.iters = trial;
                        t.xcd_chunks = xcd;
                        int grid = int(std::min<int64_t>({int64_t(wpc) * dev_cu, total, int64_t(kBarMaxGrid)}));
                        DN_HIP(hipEventRecord(e0, st));
                        if ((rc = launch_direct(st, t, grid, nt))) return rc;
                        DN_HIP(hipEventRecord(e1, st));
                        DN_HIP(hipEventSynchronize(e1));
                        if ((rc = check_err(v0, st, t.err))) return rc;
                        float ms = 0;
                        DN_HIP(hipEventElapsedTime(&ms, e0, e1));
                        if (getenv("DN_VERBOSE"))
                            fprintf(stderr, "[denser] batch tune: nt %d wpc %d xcd %d pool %d: %.3f ms\n", nt, wpc,
                                    xcd, pool, ms);
                        if (ms < best) { best = ms; ch = TuneChoice{nt, wpc, xcd, pool}; }
                    }
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        g_tuned[key] = ch;
        for (int i = 0; i < n; ++i) {
            hipStream_t keep = vols[i]->stream;
            vols[i]->stream = st;
            rc = zero_state(vols[i]);
            vols[i]->stream = keep;
            if (rc) return rc;
        }
    }
    if ((rc = build_items(ch.pool))) return rc;
    a.iters = prm->iters;
    a.xcd_chunks = ch.xcd;
    const int grid = int(std::max<int64_t>(
        1, std::min<int64_t>({int64_t(ch.wg_per_cu) * dev_cu, total, int64_t(kBarMaxGrid)})));
    hipEvent_t e0, e1;
    DN_HIP(hipEventCreate(&e0));
    DN_HIP(hipEventCreate(&e1));
    DN_HIP(hipEventRecord(e0, st));
    if (total > 0 && prm->iters > 0) {
        if ((rc = launch_graph(c, st, a, grid, ch.nt))) return rc;
    }
    DN_HIP(hipEventRecord(e1, st));
    DN_HIP(hipEventSynchronize(e1));
    float ms = 0;
    DN_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if ((rc = check_err(v0, st, a.err))) return rc;
    if (prm->gamma > 0.0)
        for (int k = 0; k < prm->iters; ++k) {
            const double th = 1.0 / std::sqrt(1.0 + 2.0 * prm->gamma * v0->acc_tau);
            v0->acc_tau = th * v0->acc_tau;
            v0->acc_sigma = v0->acc_sigma / th;
        }
    for (int i = 0; i < n; ++i) {
        dn_volume *v = vols[i];
        v->cur = (v->cur + prm->iters) & 1;
        hipStream_t keep = v->stream;
        v->stream = st;
        double ed[2] = {0, 0};
        rc = energy_current(v, prm->lambda, true, prm->data_term);
        if (!rc) rc = read_energy(v, ed);
        v->stream = keep;
        if (rc) return rc;
        if (out) {
            dn_reg_stats &s = out[i];
            s = dn_reg_stats{};
            s.energy = ed[0];
            s.dual = ed[1];
            s.gap = ed[0] - ed[1];
            s.rel_gap = ed[0] != 0.0 ? s.gap / ed[0] : 0.0;
            s.iters_run = prm->iters;
            s.converged = prm->gap_tol > 0 && s.gap <= prm->gap_tol * ed[0];
            s.ms_loop = ms;
            s.kernel_used = ch.nt * 100 + ch.wg_per_cu;
            s.layout_used = (ch.pool ? 1 : 0) | (ch.xcd ? 0 : 2);
        }
    }
    return DN_OK;
}
