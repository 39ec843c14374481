/* Test-only driver: runs the CPU oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_oracle_sanitized.py).
 * Every message sits in a heap block of exactly its length, so a read past a
 * message's last byte is reported.  Checks: one-shot equals streaming for
 * random chunkings at lengths 0..300 and a few long ones; the 64/128-bit
 * outputs are prefixes of the 256-bit one; the threaded batch driver equals
 * one-shot.  Exit status 0 only if every check holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

uint64_t hh_ref_hash64(const uint64_t key[4], const uint8_t* p, size_t len);
void hh_ref_hash128(const uint64_t key[4], const uint8_t* p, size_t len, uint64_t out[2]);
void hh_ref_hash256(const uint64_t key[4], const uint8_t* p, size_t len, uint64_t out[4]);
size_t hh_ref_cat_size(void);
struct hh_ref_cat_opaque;
void hh_ref_cat_init(void* c, const uint64_t key[4]);
void hh_ref_cat_append(void* c, const uint8_t* p, size_t len);
void hh_ref_cat_finish(const void* c, int width_words, uint64_t* out);
int hh_ref_batch(const uint64_t* keys, const uint32_t* key_idx, const uint8_t* data,
                 const uint64_t* offsets, const uint64_t* lengths, uint64_t n, int width_words,
                 uint64_t* out, int n_threads);

static uint64_t rng_state = 0x5eed1612ULL;
static uint64_t next64(void) { /* SplitMix64 */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static int failures = 0;
#define CHECK(cond, ...) do { if (!(cond)) { fprintf(stderr, __VA_ARGS__); fputc('\n', stderr); ++failures; } } while (0)

static void check_length(size_t len) {
    uint64_t key[4], one[4], h128[2], cat_out[4];
    for (int i = 0; i < 4; ++i) key[i] = next64();
    uint8_t* msg = (uint8_t*)malloc(len ? len : 1);
    for (size_t i = 0; i < len; ++i) msg[i] = (uint8_t)next64();
    hh_ref_hash256(key, msg, len, one);
    CHECK(hh_ref_hash64(key, msg, len) == one[0], "len %zu: H64 is not lane 0 of H256", len);
    hh_ref_hash128(key, msg, len, h128);
    CHECK(h128[0] == one[0] && h128[1] == one[1], "len %zu: H128 is not a prefix of H256", len);
    for (int trial = 0; trial < 3; ++trial) {
        void* cat = malloc(hh_ref_cat_size());
        hh_ref_cat_init(cat, key);
        size_t pos = 0;
        while (pos < len) {
            size_t chunk = trial == 0 ? 1 : (size_t)(next64() % 70) + 1;
            if (chunk > len - pos) chunk = len - pos;
            /* each chunk in a block of its own exact size */
            uint8_t* piece = (uint8_t*)malloc(chunk);
            memcpy(piece, msg + pos, chunk);
            hh_ref_cat_append(cat, piece, chunk);
            free(piece);
            pos += chunk;
        }
        hh_ref_cat_finish(cat, 4, cat_out);
        CHECK(memcmp(cat_out, one, sizeof one) == 0, "len %zu trial %d: streaming != one-shot", len, trial);
        free(cat);
    }
    free(msg);
}

static void check_batch(void) {
    enum { N = 97 };
    uint64_t keys[3 * 4], offsets[N], lengths[N], total = 0;
    uint32_t key_idx[N];
    for (int i = 0; i < 12; ++i) keys[i] = next64();
    for (int j = 0; j < N; ++j) {
        lengths[j] = next64() % 700;
        offsets[j] = total;
        total += lengths[j];
        key_idx[j] = (uint32_t)(next64() % 3);
    }
    uint8_t* data = (uint8_t*)malloc(total ? total : 1);
    for (uint64_t i = 0; i < total; ++i) data[i] = (uint8_t)next64();
    uint64_t* out = (uint64_t*)malloc(sizeof(uint64_t) * 2 * N);
    CHECK(hh_ref_batch(keys, key_idx, data, offsets, lengths, N, 2, out, 4) == 0, "batch failed");
    for (int j = 0; j < N; ++j) {
        uint64_t h[2];
        hh_ref_hash128(keys + 4 * key_idx[j], data + offsets[j], (size_t)lengths[j], h);
        CHECK(out[2 * j] == h[0] && out[2 * j + 1] == h[1], "batch message %d differs", j);
    }
    free(out);
    free(data);
}

int main(void) {
    for (size_t len = 0; len <= 300; ++len) check_length(len);
    const size_t longer[] = {1023, 1024, 1025, 4096 + 31, 65536 + 9};
    for (size_t i = 0; i < sizeof longer / sizeof longer[0]; ++i) check_length(longer[i]);
    check_batch();
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle sanitized: all checks passed\n");
    return 0;
}
