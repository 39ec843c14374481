// hh_api.hip -- the C ABI declared in include/hh.h: argument checks, device
// checks and dispatch to the kernel launchers.

#include <atomic>
#include <mutex>
#include <string.h>

#include "hh_device.hpp"
#include "hh_internal.hpp"

namespace hh {

namespace {

std::mutex g_mutex;
constexpr int kMaxDevices = 64;
// 0 unknown, 1 gfx950, -1 other; atomic: calls may come from several threads
std::atomic<signed char> g_device_ok[kMaxDevices];
hh_tuning g_tuning = {128u, 4u, 0u, 72u, 1u};

hh_status check_hash_args(const HashArgs& a) {
    if (a.n == 0) return HH_OK;
    if (!a.keys || a.n_keys == 0 || !a.offsets || !a.lengths || !a.out) return HH_ERR_INVALID_ARG;
    if (!a.data && a.data_bytes != 0) return HH_ERR_INVALID_ARG;
    if (a.width != 1 && a.width != 2 && a.width != 4) return HH_ERR_INVALID_ARG;
    return HH_OK;
}

}  // namespace

hh_status check_device(int* device_out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        return HH_ERR_UNSUPPORTED_DEVICE;
    }
    if (device_out) *device_out = dev;
    if (dev < kMaxDevices) {
        const signed char known = g_device_ok[dev].load(std::memory_order_relaxed);
        if (known != 0) return known > 0 ? HH_OK : HH_ERR_UNSUPPORTED_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return HH_ERR_UNSUPPORTED_DEVICE;
    }
    const bool ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    if (dev < kMaxDevices) g_device_ok[dev].store(ok ? 1 : -1, std::memory_order_relaxed);
    return ok ? HH_OK : HH_ERR_UNSUPPORTED_DEVICE;
}

hh_tuning current_tuning() {
    std::lock_guard<std::mutex> lock(g_mutex);
    return g_tuning;
}

static hh_status hash_dispatch(hh_path path, const HashArgs& a, void* stream) {
    hh_status s = check_hash_args(a);
    if (s != HH_OK || a.n == 0) return s;
    if ((s = check_device(nullptr)) != HH_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    switch (path) {
        case HH_PATH_LANE1: return launch_thread(a, 0, st);
        case HH_PATH_LANE4: return launch_quad(a, st);
        case HH_PATH_AUTO:
        case HH_PATH_BUCKETED: return launch_bucketed(a, st);
        default: return HH_ERR_INVALID_ARG;
    }
}

}  // namespace hh

using hh::HashArgs;

extern "C" {

const char* hh_status_string(hh_status status) {
    switch (status) {
        case HH_OK: return "ok";
        case HH_ERR_INVALID_ARG: return "invalid argument";
        case HH_ERR_UNSUPPORTED_DEVICE: return "no gfx950 device is current";
        case HH_ERR_OUT_OF_MEMORY: return "out of device memory";
        case HH_ERR_LAUNCH: return "kernel launch failed";
        case HH_ERR_BUSY: return "queue full, try again later";
    }
    return "unknown status";
}

int hh_version(void) { return 100; }

void hh_get_constants(uint64_t c0[4], uint64_t c1[4]) {
    for (int i = 0; i < 4; ++i) {
        c0[i] = hh::init0(i);
        c1[i] = hh::init1(i);
    }
}

hh_status hh_hash_path(hh_path path, uint32_t width_words, const uint64_t* keys, uint32_t n_keys,
                       const uint32_t* key_idx, const uint8_t* data, uint64_t data_bytes,
                       const uint64_t* offsets, const uint64_t* lengths, uint64_t n_msgs,
                       uint64_t* out, void* stream) {
    const HashArgs a{keys, n_keys, key_idx, data, data_bytes, offsets, lengths, n_msgs, out,
                     width_words};
    return hh::hash_dispatch(path, a, stream);
}

hh_status hh_hash_noalloc(uint32_t width_words, const uint64_t* keys, uint32_t n_keys,
                          const uint32_t* key_idx, const uint8_t* data, uint64_t data_bytes,
                          const uint64_t* offsets, const uint64_t* lengths, uint64_t n_msgs,
                          uint64_t* out, void* stream) {
    const HashArgs a{keys, n_keys, key_idx, data, data_bytes, offsets, lengths, n_msgs, out,
                     width_words};
    hh_status s = hh::check_hash_args(a);
    if (s != HH_OK || a.n == 0) return s;
    if (a.n > HH_NOALLOC_MAX_MSGS) return HH_ERR_INVALID_ARG;
    if ((s = hh::check_device(nullptr)) != HH_OK) return s;
    return hh::launch_bucketed_noalloc(a, (hipStream_t)stream);
}

hh_status hh_hash64(const uint64_t* keys, uint32_t n_keys, const uint32_t* key_idx,
                    const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                    const uint64_t* lengths, uint64_t n_msgs, uint64_t* out, void* stream) {
    return hh_hash_path(HH_PATH_AUTO, 1, keys, n_keys, key_idx, data, data_bytes, offsets, lengths,
                        n_msgs, out, stream);
}

hh_status hh_hash128(const uint64_t* keys, uint32_t n_keys, const uint32_t* key_idx,
                     const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                     const uint64_t* lengths, uint64_t n_msgs, uint64_t* out, void* stream) {
    return hh_hash_path(HH_PATH_AUTO, 2, keys, n_keys, key_idx, data, data_bytes, offsets, lengths,
                        n_msgs, out, stream);
}

hh_status hh_hash256(const uint64_t* keys, uint32_t n_keys, const uint32_t* key_idx,
                     const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                     const uint64_t* lengths, uint64_t n_msgs, uint64_t* out, void* stream) {
    return hh_hash_path(HH_PATH_AUTO, 4, keys, n_keys, key_idx, data, data_bytes, offsets, lengths,
                        n_msgs, out, stream);
}

hh_status hh_hash64_uniform(const uint64_t* keys, uint32_t n_keys, const uint32_t* key_idx,
                            const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                            uint64_t length, uint64_t n_msgs, uint64_t* out, void* stream) {
    if (n_msgs == 0) return HH_OK;
    if (!keys || n_keys == 0 || !offsets || !out || (!data && data_bytes != 0))
        return HH_ERR_INVALID_ARG;
    hh_status s = hh::check_device(nullptr);
    if (s != HH_OK) return s;
    const HashArgs a{keys, n_keys, key_idx, data, data_bytes, offsets, nullptr, n_msgs, out, 1};
    return hh::launch_thread(a, length, (hipStream_t)stream);
}

hh_status hh_prf(uint32_t width_words, const uint64_t* keys, uint32_t n_keys,
                 uint64_t counter_base, uint64_t n, uint64_t* out, void* stream) {
    if (n == 0) return HH_OK;
    if (!keys || n_keys == 0 || !out) return HH_ERR_INVALID_ARG;
    if (width_words != 1 && width_words != 2 && width_words != 4) return HH_ERR_INVALID_ARG;
    hh_status s = hh::check_device(nullptr);
    if (s != HH_OK) return s;
    return hh::launch_prf(width_words, keys, n_keys, counter_base, n, out, (hipStream_t)stream);
}

hh_status hh_state_init(const uint64_t* keys, uint32_t n_keys, const uint32_t* key_idx,
                        uint64_t* states, uint64_t n_states, const uint32_t* state_idx, uint64_t n,
                        void* stream) {
    if (n == 0) return HH_OK;
    if (!keys || n_keys == 0 || !states) return HH_ERR_INVALID_ARG;
    hh_status s = hh::check_device(nullptr);
    if (s != HH_OK) return s;
    return hh::launch_state_init(keys, n_keys, key_idx, states, n_states, state_idx, n,
                                 (hipStream_t)stream);
}

hh_status hh_copy_segments(uint8_t* dst, uint64_t dst_bytes, const uint8_t* src,
                           uint64_t src_bytes, const uint64_t* src_offs, const uint64_t* dst_offs,
                           const uint64_t* lens, uint64_t n, uint64_t max_len, void* stream) {
    if (n == 0) return HH_OK;
    if (!dst || !src || !src_offs || !dst_offs || !lens) return HH_ERR_INVALID_ARG;
    hh_status s = hh::check_device(nullptr);
    if (s != HH_OK) return s;
    return hh::launch_copy_segments(dst, dst_bytes, src, src_bytes, src_offs, dst_offs, lens, n,
                                    max_len, (hipStream_t)stream);
}

hh_status hh_state_update(uint64_t* states, uint64_t n_states, const uint32_t* state_idx,
                          const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                          const uint64_t* lengths, uint64_t n, void* stream) {
    if (n == 0) return HH_OK;
    if (!states || !offsets || !lengths || (!data && data_bytes != 0)) return HH_ERR_INVALID_ARG;
    hh_status s = hh::check_device(nullptr);
    if (s != HH_OK) return s;
    return hh::launch_state_step(0, states, n_states, state_idx, data, data_bytes, offsets,
                                 lengths, nullptr, nullptr, 0, nullptr, n, (hipStream_t)stream);
}

hh_status hh_state_final(uint64_t* states, uint64_t n_states, const uint32_t* state_idx,
                         const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                         const uint64_t* lengths, const uint8_t* width_words, uint64_t* out,
                         uint64_t out_words, const uint64_t* out_offsets, uint64_t n,
                         void* stream) {
    if (n == 0) return HH_OK;
    if (!states || !offsets || !lengths || !out || (!data && data_bytes != 0))
        return HH_ERR_INVALID_ARG;
    hh_status s = hh::check_device(nullptr);
    if (s != HH_OK) return s;
    return hh::launch_state_step(1, states, n_states, state_idx, data, data_bytes, offsets,
                                 lengths, width_words, out, out_words, out_offsets, n,
                                 (hipStream_t)stream);
}

hh_status hh_state_step(uint64_t* states, uint64_t n_states, const uint32_t* state_idx,
                        const uint8_t* data, uint64_t data_bytes, const uint64_t* offsets,
                        const uint64_t* lengths, const uint8_t* width_words, uint64_t* out,
                        uint64_t out_words, const uint64_t* out_offsets, uint64_t n,
                        void* stream) {
    if (n == 0) return HH_OK;
    if (!states || !offsets || !lengths || !width_words || (!data && data_bytes != 0))
        return HH_ERR_INVALID_ARG;
    hh_status s = hh::check_device(nullptr);
    if (s != HH_OK) return s;
    return hh::launch_state_step(2, states, n_states, state_idx, data, data_bytes, offsets,
                                 lengths, width_words, out, out ? out_words : 0, out_offsets, n,
                                 (hipStream_t)stream);
}

hh_status hh_avalanche(int mode, uint32_t msg_bytes, uint32_t rounds, uint64_t seed,
                       const uint64_t key[4], uint64_t n_samples, uint32_t bit_first,
                       uint32_t bit_count, uint64_t* counts, void* stream) {
    if (n_samples == 0) return HH_OK;
    if ((mode != 0 && mode != 1) || msg_bytes < 1 || msg_bytes > 32 || rounds < 1 ||
        rounds > 4 || bit_count < 1 || bit_count > 32 || !counts ||
        (uint64_t)bit_first + bit_count > 8ull * msg_bytes || (mode == 1 && !key))
        return HH_ERR_INVALID_ARG;
    hh_status s = hh::check_device(nullptr);
    if (s != HH_OK) return s;
    return hh::launch_avalanche(mode, msg_bytes, rounds, seed, key, n_samples, bit_first,
                                bit_count, counts, (hipStream_t)stream);
}

void hh_get_tuning(hh_tuning* t) {
    if (t) *t = hh::current_tuning();
}

hh_status hh_set_tuning(const hh_tuning* t) {
    if (!t || t->waves_per_cu == 0 || t->waves_per_cu > 32 || t->use_graph > 1 ||
        t->isolate_long > 1)
        return HH_ERR_INVALID_ARG;
    if (t->long_ring != 36 && t->long_ring != 48 && t->long_ring != 72 && t->long_ring != 96)
        return HH_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(hh::g_mutex);
    hh::g_tuning = *t;
    return HH_OK;
}

hh_status hh_pinned_device_pointer(const void* host, void** device) {
    if (!host || !device) return HH_ERR_INVALID_ARG;
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, const_cast<void*>(host), 0) != hipSuccess || !d) {
        (void)hipGetLastError();
        return HH_ERR_INVALID_ARG;
    }
    *device = d;
    return HH_OK;
}

hh_status hh_release(void) {
    hh::release_bucketed();
    return HH_OK;
}

hh_status hh_timing_enable(int enable) { return hh::timing_enable(enable != 0); }

hh_status hh_timing_collect(uint32_t* launches, double* total_ms) {
    return hh::timing_collect(launches, total_ms);
}

}  // extern "C"
