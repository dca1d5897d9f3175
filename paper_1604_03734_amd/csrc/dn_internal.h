// Internal declarations of the denser HIP library (gfx950).  Not part of
// the public ABI (include/denser.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "denser.h"

namespace dn {

constexpr int kBlockVox = 512;     // 8^3 voxels per block
constexpr int kNbr = 27;           // 3x3x3 neighbourhood, centre = self
constexpr int kCentre = 13;

void set_error(const char *fmt, ...);

#define DN_HIP(expr)                                                           \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) {                                                \
            ::dn::set_error("%s failed: %s (%s:%d)", #expr,                    \
                            hipGetErrorString(e_), __FILE__, __LINE__);        \
            return DN_E_DEVICE;                                                \
        }                                                                      \
    } while (0)

#define DN_REQUIRE(cond, ...)                                                  \
    do {                                                                       \
        if (!(cond)) {                                                         \
            ::dn::set_error(__VA_ARGS__);                                      \
            return DN_E_INVALID;                                               \
        }                                                                      \
    } while (0)

// Bump allocator over caller-owned device memory.  With a null base it
// only measures (the same sequence of take() calls sizes a region and later
// carves it, so sizing and use cannot disagree).  Every piece starts on a
// 256-byte boundary.
struct Bump {
    char *base;
    size_t cap;
    size_t off = 0;
    Bump(void *b, size_t c) : base(static_cast<char *>(b)), cap(c) {}
    template <class T> T *take(size_t n)
    {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
    bool fits() const { return off <= cap; }
};

// Temporary storage handed to the rocprim calls: a bound on what they ask
// for (a radix sort needs one copy of its keys and values plus small
// tables, the scans, selections and reductions a few bytes per thousand
// items), so every scratch region is sized before the first call.  rocprim
// checks the size it is given and fails (no write) if it needed more; the
// library also compares the bounds with rocprim's own figures once per
// volume.
inline size_t tmp_sort(size_t n, size_t key_value_bytes) { return n * key_value_bytes + n / 2 + (size_t(2) << 20); }
inline size_t tmp_light(size_t n) { return n / 16 + (size_t(1) << 20); }

// The scratch buffers of one insertion of n_cand candidate keys into a
// pool that will hold at most n_blocks blocks (volume.hip).
struct InsertScratch {
    uint8_t *flags;
    uint64_t *newraw, *sorted, *newk, *ksorted;
    int32_t *pos0, *pos1;               // candidate positions (order-keeping insertion)
    int32_t *ids0, *ids1;
    uint32_t *home, *home2;
    int64_t *dm, *runmax;
    void *tmp;
    size_t tmp_bytes;
};
InsertScratch carve_insert(Bump &b, int64_t n_cand, int64_t n_blocks);

}  // namespace dn

// The opaque volume handle.
struct dn_volume {
    dn_volume_params prm{};
    hipStream_t stream = nullptr;
    int device = 0;
    int64_t nb = 0;              // allocated blocks
    int64_t cap_blocks = 0;      // max_blocks
    int64_t hash_slots = 0;      // cap + tail
    uint32_t hash_cap = 0;

    // block pool
    int32_t *coords = nullptr;   // [max][4] x, y, z, 0
    uint64_t *keys = nullptr;    // [max] packed keys, pool order
    int32_t *hash[2] = {nullptr, nullptr};  // [slots][4], double buffered
    int cur_hash = 0;
    int32_t *nbr = nullptr;      // [max][27]

    // fused data
    float *f = nullptr, *w = nullptr;   // [max][512]

    // solver state, FP32: u in place; ubar and p ping-pong for the fused kernel
    float *u = nullptr;
    float *ubar[2] = {nullptr, nullptr};
    float *p[2] = {nullptr, nullptr};   // each [3][max][512]
    int cur = 0;                        // index of the current ubar/p buffers
    // 16-bit solver state (in the arena when the volume has state16)
    void *u16 = nullptr;
    void *ubar16[2] = {nullptr, nullptr};
    void *p16[2] = {nullptr, nullptr};
    int state_storage = DN_F32;         // where the current state lives
    uint64_t lowp_iter = 0;             // 16-bit iterations run (seeds the stochastic rounding)
    double acc_tau = 0, acc_sigma = 0;  // accelerated schedule (tau_n, sigma_n)
    int64_t nb_state = 0;               // blocks whose solver state a regularize call set

    uint8_t *emask = nullptr;           // [max][512]
    int64_t emask_nb = -1;              // nb for which emask/order are valid
    int32_t *order = nullptr;           // [max] processing order (Morton)
    int layout = 0;                     // chosen by the autotuner, see regularize.hip
    double *partials = nullptr;         // [max][2]
    double *energy2 = nullptr;          // [2] device

    // caller-owned arena: everything above lives in it, then
    void *arena = nullptr;
    size_t arena_bytes = 0;
    uint64_t *cand = nullptr;           // [max_candidates] raw candidate keys of the last frame
    int64_t cand_n = 0;                 // how many the last allocation call listed
    int64_t *misc = nullptr;            // small device counters (256 bytes)
    char *scratch = nullptr;            // per-call scratch, reused by every call
    size_t scratch_bytes = 0;
    int64_t host_stage[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // host side of small read-backs
};

namespace dn {
// regularize.hip
int build_masks(dn_volume *v);
size_t masks_scratch(int64_t n_blocks);
// volume.hip
int build_candidates(dn_volume *v, uint64_t **uniq, int64_t *n_uniq);
size_t candidates_scratch(int64_t n_cand);
int zero_state(dn_volume *v);
int energy_current(dn_volume *v, double lambda, bool use_f32, int data_term);
int read_energy(dn_volume *v, double out[2]);
int reduce_pairs(dn_volume *v, int64_t n);
// volume.hip
int volume_sync(dn_volume *v);
int read_back(dn_volume *v, const void *dev, size_t bytes);   // into v->host_stage, synchronises
// extract.hip
size_t extract_scratch(int64_t n_blocks);
}  // namespace dn
