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

// A device buffer that only grows.
struct Buf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t need);   // DN_OK or DN_E_DEVICE
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Pinned host staging for small read-backs.
struct HostBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t need);
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

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
    // 16-bit solver state (allocated on first use)
    void *u16 = nullptr;
    void *ubar16[2] = {nullptr, nullptr};
    void *p16[2] = {nullptr, nullptr};
    int state_storage = DN_F32;         // where the current state lives
    double acc_tau = 0, acc_sigma = 0;  // accelerated schedule (tau_n, sigma_n)
    int64_t nb_state = 0;               // blocks whose solver state a regularize call set

    uint8_t *emask = nullptr;           // [max][512]
    int64_t emask_nb = -1;              // nb for which emask/order are valid
    int32_t *order = nullptr;           // [max] processing order (Morton)
    int layout = 0;                     // chosen by the autotuner, see regularize.hip
    double *partials = nullptr;         // [max][2]
    double *energy2 = nullptr;          // [2] device

    // scratch for allocation and extraction
    dn::Buf s_cand, s_cand2, s_counts, s_offsets, s_tmp, s_uniq, s_flags, s_new, s_sorted,
        s_vals, s_vals2, s_home, s_home2, s_pos, s_misc, s_laser;
    dn::Buf s_newk;                     // distinct new keys of an insertion
    int64_t last_nuniq = 0;             // distinct candidates of the last frame (once built)
    const uint64_t *cand_src = nullptr; // raw candidate list of the last frame
    int64_t cand_n = 0;
    bool cand_pending = false;          // its distinct list is not built yet
    dn::HostBuf host;
};

namespace dn {
// regularize.hip
int build_masks(dn_volume *v);
// volume.hip
int ensure_candidates(dn_volume *v);
int ensure_lowp(dn_volume *v);
int zero_state(dn_volume *v);
int energy_current(dn_volume *v, double lambda, bool use_f32, int data_term);
int read_energy(dn_volume *v, double out[2]);
int reduce_pairs(dn_volume *v, int64_t n);
// volume.hip
int volume_sync(dn_volume *v);
}  // namespace dn
