/* Test-only driver: the finalization-round study of Sec. 4.3 on the CPU.
 *
 * All 2^24 three-byte inputs are hashed under one key with 1..R finalization
 * rounds; for every (input bit b, output bit o) the probability p that output
 * bit o of the 64-bit hash toggles when input bit b flips is counted over the
 * 2^23 input pairs that differ in bit b.  Printed per round count: the mean
 * and the max over the 24 x 64 cells of |2p - 1|.
 *
 * Variant "oracle" runs the oracle's own remainder step (hh_ref_remainder).
 * The other variants are alternative readings of the Sec. 4.5 padding text,
 * built here from the oracle's Reset, Update and Permute; they exist only for
 * this study and are never part of the oracle or of the library:
 *   placement of the last r%4 tail bytes (the whole 4-byte groups always go
 *   to packet bytes 0..q-1):
 *     t28  packet bytes 28.. (top dword of the 32-byte packet)
 *     t29  packet bytes 32-m..31 (top bytes of the packet)
 *     half top dword of the 16-byte half that holds byte q: bytes 12.. when
 *          r < 16, bytes 28.. when r >= 16
 *     h13  as half, but the top m bytes of that dword (16-m.. / 32-m..)
 *     t20  bytes 20.. (top dword of lane 2)
 *     t4   bytes 4.. (top dword of lane 0)
 *     cont right after the whole groups (bytes q..q+m-1)
 *   rotation of each 32-bit half of v1 by r: L (left) or R (right);
 *   size injection: 64 (one 64-bit add of r*(2^32+1)) or 32 (two 32-bit adds,
 *   no carry between the halves).
 * A variant is written placement/rotation/injection, e.g. "half/L/64".
 *
 * usage: rounds_study key0 key1 key2 key3 max_rounds threads variant...
 * (key words in hex).  Output: "variant rounds mean_bias max_bias" lines,
 * biases as fractions. */
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t v0[4], v1[4], mul0[4], mul1[4];
} study_state; /* the oracle's state layout */

void hh_ref_reset(const uint64_t key[4], study_state* s);
void hh_ref_update(study_state* s, const uint64_t packet[4]);
void hh_ref_permute(const uint64_t v0[4], uint64_t out[4]);
void hh_ref_remainder(study_state* s, const uint8_t* tail, size_t r);

enum { IN_BYTES = 3, IN_BITS = 8 * IN_BYTES, MAX_ROUNDS = 8, MAX_THREADS = 64 };
#define N_INPUTS (1u << IN_BITS)

typedef struct {
    int oracle;    /* 1: use hh_ref_remainder */
    char place[8]; /* t28 t29 half h13 t20 t4 cont */
    int rot_left;
    int inject64;
} variant;

static uint64_t g_key[4];
static int g_rounds;
static variant g_var;
static uint64_t* g_hash[MAX_ROUNDS + 1]; /* g_hash[k][x]: lane-0 sum after k rounds */

static uint32_t rotl32(uint32_t x, unsigned r) { return (x << r) | (x >> (32 - r)); }
static uint32_t rotr32(uint32_t x, unsigned r) { return (x >> r) | (x << (32 - r)); }

/* start byte of the last m = r%4 tail bytes under the variant's placement */
static size_t tail_slot(const char* place, size_t r, size_t q, size_t m) {
    if (!strcmp(place, "t28")) return 28;
    if (!strcmp(place, "t29")) return 32 - m;
    if (!strcmp(place, "half")) return r < 16 ? 12 : 28;
    if (!strcmp(place, "h13")) return r < 16 ? 16 - m : 32 - m;
    if (!strcmp(place, "t20")) return 20;
    if (!strcmp(place, "t4")) return 4;
    return q; /* cont */
}

static void variant_remainder(study_state* s, const uint8_t* tail, size_t r) {
    if (g_var.oracle) {
        hh_ref_remainder(s, tail, r);
        return;
    }
    const size_t q = r - r % 4, m = r % 4;
    for (int i = 0; i < 4; ++i) {
        uint32_t lo = (uint32_t)s->v0[i], hi = (uint32_t)(s->v0[i] >> 32);
        if (g_var.inject64) {
            s->v0[i] += ((uint64_t)r << 32) | r;
        } else {
            lo += (uint32_t)r;
            hi += (uint32_t)r;
            s->v0[i] = ((uint64_t)hi << 32) | lo;
        }
        lo = (uint32_t)s->v1[i];
        hi = (uint32_t)(s->v1[i] >> 32);
        if (g_var.rot_left) {
            lo = rotl32(lo, (unsigned)r);
            hi = rotl32(hi, (unsigned)r);
        } else {
            lo = rotr32(lo, (unsigned)r);
            hi = rotr32(hi, (unsigned)r);
        }
        s->v1[i] = ((uint64_t)hi << 32) | lo;
    }
    uint8_t P[32];
    memset(P, 0, sizeof P);
    for (size_t j = 0; j < q; ++j) P[j] = tail[j];
    const size_t slot = tail_slot(g_var.place, r, q, m);
    for (size_t j = 0; j < m; ++j) P[slot + j] = tail[q + j];
    uint64_t packet[4];
    for (int i = 0; i < 4; ++i) {
        uint64_t w = 0;
        for (int j = 7; j >= 0; --j) w = (w << 8) | P[8 * i + j];
        packet[i] = w;
    }
    hh_ref_update(s, packet);
}

typedef struct {
    uint32_t begin, end;
    uint64_t cnt[MAX_ROUNDS + 1][IN_BITS][64];
} job;

static void* hash_range(void* arg) {
    job* J = (job*)arg;
    for (uint32_t x = J->begin; x < J->end; ++x) {
        study_state s;
        uint8_t msg[IN_BYTES];
        for (int j = 0; j < IN_BYTES; ++j) msg[j] = (uint8_t)(x >> (8 * j));
        hh_ref_reset(g_key, &s);
        variant_remainder(&s, msg, IN_BYTES);
        for (int k = 1; k <= g_rounds; ++k) {
            uint64_t pk[4];
            hh_ref_permute(s.v0, pk);
            hh_ref_update(&s, pk);
            g_hash[k][x] = s.v0[0] + s.v1[0] + s.mul0[0] + s.mul1[0];
        }
    }
    return NULL;
}

/* flip counts over the pairs (x, x | 1<<b) with bit b of x clear and x in the
 * job's range; bits of the xor are accumulated eight at a time in byte-wide
 * counters (bit 8t+j of d in byte t of acc[j]) and flushed before they wrap */
static void* count_range(void* arg) {
    job* J = (job*)arg;
    for (int k = 1; k <= g_rounds; ++k) {
        const uint64_t* H = g_hash[k];
        for (int b = 0; b < IN_BITS; ++b) {
            const uint32_t bit = 1u << b;
            uint64_t acc[8] = {0};
            int pending = 0;
            for (uint32_t x = J->begin; x < J->end; ++x) {
                if (x & bit) continue;
                const uint64_t d = H[x] ^ H[x | bit];
                for (int j = 0; j < 8; ++j) acc[j] += (d >> j) & 0x0101010101010101ULL;
                if (++pending == 255) {
                    for (int j = 0; j < 8; ++j)
                        for (int t = 0; t < 8; ++t) J->cnt[k][b][8 * t + j] += (acc[j] >> (8 * t)) & 0xff;
                    memset(acc, 0, sizeof acc);
                    pending = 0;
                }
            }
            for (int j = 0; j < 8; ++j)
                for (int t = 0; t < 8; ++t) J->cnt[k][b][8 * t + j] += (acc[j] >> (8 * t)) & 0xff;
        }
    }
    return NULL;
}

static int parse_variant(const char* text, variant* v) {
    memset(v, 0, sizeof *v);
    if (!strcmp(text, "oracle")) {
        v->oracle = 1;
        return 0;
    }
    char place[16], rot;
    int inj;
    if (sscanf(text, "%7[a-z0-9]/%c/%d", place, &rot, &inj) != 3) return 1;
    static const char* names[] = {"t28", "t29", "half", "h13", "t20", "t4", "cont"};
    int ok = 0;
    for (size_t i = 0; i < sizeof names / sizeof names[0]; ++i) ok |= !strcmp(place, names[i]);
    if (!ok || (rot != 'L' && rot != 'R') || (inj != 64 && inj != 32)) return 1;
    strcpy(v->place, place);
    v->rot_left = rot == 'L';
    v->inject64 = inj == 64;
    return 0;
}

int main(int argc, char** argv) {
    if (argc < 8) {
        fprintf(stderr, "usage: %s key0 key1 key2 key3 max_rounds threads variant...\n", argv[0]);
        return 2;
    }
    for (int i = 0; i < 4; ++i) g_key[i] = strtoull(argv[1 + i], NULL, 16);
    g_rounds = atoi(argv[5]);
    int threads = atoi(argv[6]);
    if (g_rounds < 1 || g_rounds > MAX_ROUNDS || threads < 1 || threads > MAX_THREADS) return 2;
    for (int k = 1; k <= g_rounds; ++k) {
        g_hash[k] = (uint64_t*)malloc(sizeof(uint64_t) * N_INPUTS);
        if (!g_hash[k]) return 3;
    }
    job* jobs = (job*)calloc((size_t)threads, sizeof(job));
    if (!jobs) return 3;
    pthread_t tid[MAX_THREADS];
    for (int a = 7; a < argc; ++a) {
        if (parse_variant(argv[a], &g_var)) {
            fprintf(stderr, "bad variant %s\n", argv[a]);
            return 2;
        }
        memset(jobs, 0, sizeof(job) * (size_t)threads);
        for (int t = 0; t < threads; ++t) {
            jobs[t].begin = (uint32_t)((uint64_t)N_INPUTS * t / threads);
            jobs[t].end = (uint32_t)((uint64_t)N_INPUTS * (t + 1) / threads);
        }
        for (int t = 0; t < threads; ++t) pthread_create(&tid[t], NULL, hash_range, &jobs[t]);
        for (int t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
        for (int t = 0; t < threads; ++t) pthread_create(&tid[t], NULL, count_range, &jobs[t]);
        for (int t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
        const double pairs = (double)(N_INPUTS / 2);
        for (int k = 1; k <= g_rounds; ++k) {
            double sum = 0.0, mx = 0.0;
            for (int b = 0; b < IN_BITS; ++b)
                for (int o = 0; o < 64; ++o) {
                    uint64_t c = 0;
                    for (int t = 0; t < threads; ++t) c += jobs[t].cnt[k][b][o];
                    double dev = 2.0 * (double)c / pairs - 1.0;
                    if (dev < 0) dev = -dev;
                    sum += dev;
                    if (dev > mx) mx = dev;
                }
            printf("%s %d %.9f %.9f\n", argv[a], k, sum / (IN_BITS * 64), mx);
        }
        fflush(stdout);
    }
    for (int k = 1; k <= g_rounds; ++k) free(g_hash[k]);
    free(jobs);
    return 0;
}
