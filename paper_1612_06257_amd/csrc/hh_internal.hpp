// hh_internal.hpp -- declarations shared by the host-side translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hh.h"

namespace hh {

struct HashArgs {
    const uint64_t* keys;
    uint32_t n_keys;
    const uint32_t* key_idx;
    const uint8_t* data;
    uint64_t data_bytes;
    const uint64_t* offsets;
    const uint64_t* lengths;
    uint64_t n;
    uint64_t* out;
    uint32_t width;  // output words: 1, 2 or 4
};

hh_status launch_thread(const HashArgs& a, uint64_t uniform_length, hipStream_t st);
hh_status launch_quad(const HashArgs& a, hipStream_t st);
hh_status launch_bucketed(const HashArgs& a, hipStream_t st);
hh_status launch_bucketed_noalloc(const HashArgs& a, hipStream_t st);
hh_status launch_prf(uint32_t width, const uint64_t* keys, uint32_t n_keys, uint64_t counter_base,
                     uint64_t n, uint64_t* out, hipStream_t st);
hh_status launch_state_init(const uint64_t* keys, uint32_t n_keys, const uint32_t* key_idx,
                            uint64_t* states, uint64_t n_states, const uint32_t* state_idx,
                            uint64_t n, hipStream_t st);
hh_status launch_copy_segments(uint8_t* dst, uint64_t dst_bytes, const uint8_t* src,
                               uint64_t src_bytes, const uint64_t* src_offs,
                               const uint64_t* dst_offs, const uint64_t* lens, uint64_t n,
                               uint64_t max_len, hipStream_t st);
hh_status launch_state_step(int mode, uint64_t* states, uint64_t n_states,
                            const uint32_t* state_idx, const uint8_t* data, uint64_t data_bytes,
                            const uint64_t* offsets, const uint64_t* lengths,
                            const uint8_t* width_words, uint64_t* out, uint64_t out_words,
                            const uint64_t* out_offsets, uint64_t n, hipStream_t st);

hh_status launch_avalanche(int mode, uint32_t msg_bytes, uint32_t rounds, uint64_t seed,
                           const uint64_t key[4], uint64_t n, uint32_t bit_first,
                           uint32_t bit_count, uint64_t* counts, hipStream_t st);

// current device is a gfx950 (cached per device); HH_OK or an error status
hh_status check_device(int* device_out);

// process-wide tuning (hh_set_tuning)
hh_tuning current_tuning();

void release_bucketed();
hh_status timing_enable(bool on);
hh_status timing_collect(uint32_t* launches, double* total_ms);

}  // namespace hh
