"""The pins catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of ``oracle/hh_oracle.c`` (on the CPU),
compiles it, routes the oracle module to the broken build and runs the pins
from test_oracle_steps / test_oracle_properties / test_oracle_rounds.  At least
one pin must fail for every mistake.  The frozen golden vectors are
deliberately NOT part of the battery, nor is the test that restates the
oracle's own remainder formula: the mistakes must be caught by what the paper
fixes.  The one reading the paper leaves open (the direction of the v1
rotation) is listed in UNPINNED: its mistake is caught only by that
conformance test.
"""
import os

import pytest

import oracle
import test_oracle_properties as P
import test_oracle_rounds as R
import test_oracle_steps as S

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "hh_oracle.c")

MUTATIONS = {
    "update drops v1 += mul0": (
        "s->v1[i] = s->v1[i] + word + s->mul0[i];", "s->v1[i] = s->v1[i] + word;"),
    "update drops v0 += mul1": (
        "s->v0[i] += s->mul1[i];", ""),
    "first product operands transposed": (
        "s->mul0[i] ^= lo32(s->v1[i]) * hi32(s->v0[i]);",
        "s->mul0[i] ^= lo32(s->v0[i]) * hi32(s->v1[i]);"),
    "first product uses lo32 of v0": (
        "s->mul0[i] ^= lo32(s->v1[i]) * hi32(s->v0[i]);",
        "s->mul0[i] ^= lo32(s->v1[i]) * lo32(s->v0[i]);"),
    "second product uses hi32 of v0": (
        "s->mul1[i] ^= lo32(s->v0[i]) * hi32(s->v1[i]);",
        "s->mul1[i] ^= lo32(s->v0[i]) * hi32(s->v0[i]);"),
    "mul0 added instead of xored": (
        "s->mul0[i] ^= lo32(s->v1[i]) * hi32(s->v0[i]);",
        "s->mul0[i] += lo32(s->v1[i]) * hi32(s->v0[i]);"),
    "packet xored instead of added": (
        "s->v1[i] = s->v1[i] + word + s->mul0[i];", "s->v1[i] = (s->v1[i] ^ word) + s->mul0[i];"),
    "second zipper reads stale v0": (
        "    zipper_merge_vec(s->v1, z);\n"
        "    for (int i = 0; i < 4; ++i) s->v0[i] += z[i];\n"
        "    zipper_merge_vec(s->v0, z);\n"
        "    for (int i = 0; i < 4; ++i) s->v1[i] += z[i];",
        "    uint64_t z0[4];\n    zipper_merge_vec(s->v0, z0);\n    zipper_merge_vec(s->v1, z);\n"
        "    for (int i = 0; i < 4; ++i) s->v0[i] += z[i];\n"
        "    for (int i = 0; i < 4; ++i) s->v1[i] += z0[i];"),
    "zipper list read low-first": (
        "uint8_t P_i = HH_REF_ZIPPER_PRINTED[15 - i];", "uint8_t P_i = HH_REF_ZIPPER_PRINTED[i];"),
    "zipper pairs lanes (0,2),(1,3)": (
        "hh_ref_zipper_merge(v[0], v[1], &out[0], &out[1]);\n    hh_ref_zipper_merge(v[2], v[3], &out[2], &out[3]);",
        "hh_ref_zipper_merge(v[0], v[2], &out[0], &out[2]);\n    hh_ref_zipper_merge(v[1], v[3], &out[1], &out[3]);"),
    "permute indices read low-first": (
        "dst[e] = src[HH_REF_PERMUTE_PRINTED[7 - e]];", "dst[e] = src[HH_REF_PERMUTE_PRINTED[e]];"),
    "permute without 32-bit half swap": (
        "for (int i = 0; i < 4; ++i) out[i] = ((uint64_t)dst[2 * i + 1] << 32) | dst[2 * i];",
        "for (int i = 0; i < 4; ++i) out[i] = ((uint64_t)dst[2 * i] << 32) | dst[2 * i + 1];"),
    "reset without rot32 of the key": (
        "s->v1[i] = rot32(key[i]) ^ HH_REF_C1[i];", "s->v1[i] = key[i] ^ HH_REF_C1[i];"),
    "reset swaps mul0 and mul1": (
        "s->mul0[i] = HH_REF_C0[i];\n        s->mul1[i] = HH_REF_C1[i];",
        "s->mul0[i] = HH_REF_C1[i];\n        s->mul1[i] = HH_REF_C0[i];"),
    "constant lane 0 by OR reading": (
        "0xdbe6d5d5fe4cce2fULL", "0xdbeeffddfe4eeeafULL"),
    "little-endian packet read big-endian": (
        "for (int j = 7; j >= 0; --j) x = (x << 8) | b[j];",
        "for (int j = 0; j < 8; ++j) x = (x << 8) | b[j];"),
    "size injected into low halves only": (
        "uint64_t broadcast = ((uint64_t)r << 32) | (uint64_t)r;", "uint64_t broadcast = (uint64_t)r;"),
    "v1 halves rotated right": (
        "static uint32_t rotl32(uint32_t x, unsigned r) { return (x << r) | (x >> (32 - r)); }",
        "static uint32_t rotl32(uint32_t x, unsigned r) { return (x >> r) | (x << (32 - r)); }"),
    "trailing bytes right after the whole groups": (
        "for (size_t j = 0; j < m; ++j) P[top + j] = tail[q + j];",
        "for (size_t j = 0; j < m; ++j) P[q + j] = tail[q + j];"),
    "trailing bytes at packet bytes 28.. for every size": (
        "size_t top = r < 16 ? 12 : 28;", "size_t top = 28;"),
    "trailing bytes at packet bytes 12.. for every size": (
        "size_t top = r < 16 ? 12 : 28;", "size_t top = 12;"),
    "trailing bytes dropped": (
        "for (size_t j = 0; j < m; ++j) P[top + j] = tail[q + j];", ""),
    "v1 not rotated": (
        "uint32_t lo = rotl32((uint32_t)lo32(s->v1[i]), (unsigned)r);\n"
        "        uint32_t hi = rotl32((uint32_t)hi32(s->v1[i]), (unsigned)r);",
        "uint32_t lo = (uint32_t)lo32(s->v1[i]);\n        uint32_t hi = (uint32_t)hi32(s->v1[i]);"),
    "size injected after the padded packet's update": (
        "    hh_ref_update(s, packet);\n}",
        "    for (int i = 0; i < 4; ++i) s->v0[i] -= broadcast;\n    hh_ref_update(s, packet);\n"
        "    for (int i = 0; i < 4; ++i) s->v0[i] += broadcast;\n}"),
    "size not injected into v0": (
        "s->v0[i] += broadcast;", ""),
    "padding packet taken from the head instead of the tail": (
        "if (r != 0) hh_ref_remainder(&s, p + 32 * full, r);",
        "if (r != 0) hh_ref_remainder(&s, p, r);"),
    "padding also for multiples of 32": (
        "if (r != 0) hh_ref_remainder(&s, p + 32 * full, r);",
        "hh_ref_remainder(&s, p + 32 * full, r);"),
    "three finalization rounds": (
        "hh_ref_hash_rounds(key, p, len, 4, sum);\n    return sum[0];",
        "hh_ref_hash_rounds(key, p, len, 3, sum);\n    return sum[0];"),
    "permute result overwrites v0": (
        "hh_ref_permute(s->v0, q);\n        hh_ref_update(s, q);",
        "hh_ref_permute(s->v0, q);\n        for (int i = 0; i < 4; ++i) s->v0[i] = q[i];\n"
        "        hh_ref_update(s, q);"),
    "final sum xors": (
        "sum[i] = s->v0[i] + s->v1[i] + s->mul0[i] + s->mul1[i];",
        "sum[i] = s->v0[i] ^ s->v1[i] ^ s->mul0[i] ^ s->mul1[i];"),
    "128-bit hash takes lanes 0 and 2": (
        "out[0] = sum[0];\n    out[1] = sum[1];", "out[0] = sum[0];\n    out[1] = sum[2];"),
    "stream finish ignores the buffered bytes": (
        "if (c->n != 0) hh_ref_remainder(&s, c->buf, c->n);", ""),
}


UNPINNED = {"v1 halves rotated right"}


def _battery(zipper_printed, permute_printed, src, workdir):
    """Pins against what the paper fixes, cheapest first; the round-count
    study (a few seconds) comes last."""
    return [
        lambda: S.test_oracle_zipper_applies_printed_permutation(zipper_printed),
        lambda: S.test_oracle_permute_applies_printed_indices(permute_printed),
        lambda: S.test_permute_swaps_128bit_halves_and_32bit_halves(),
        lambda: S.test_constants_follow_pi_derivation("machin"),
        lambda: S.test_constants_set_every_bit_in_some_lane(),
        lambda: S.test_reset_expands_key(),
        lambda: S.test_update_on_zero_state_closed_form(),
        lambda: S.test_update_multiply_uses_low_v1_times_high_v0(),
        lambda: S.test_update_second_multiply_after_adding_mul1(),
        lambda: S.test_update_is_a_bijection_round_trip(),
        lambda: S.test_update_lanes_pairwise_independent(),
        lambda: S.test_remainder_adds_size_to_every_32bit_half_of_v0_before_its_update(),
        lambda: S.test_remainder_packet_holds_the_tail_and_v1_is_rotated(),
        lambda: S.test_no_remainder_step_for_multiples_of_32(),
        lambda: S.test_finalize_is_four_permute_updates_then_sum(),
        lambda: P.test_streaming_equals_one_shot(1),
        lambda: P.test_zero_messages_of_different_lengths_differ(),
        lambda: P.test_upper_half_of_packet_reaches_h64(),
        lambda: P.test_wide_outputs_share_the_final_sum(),
        lambda: P.test_two_finalization_rounds_are_biased_four_are_not(),
        lambda: R.check_rounds_figures(R.round_biases(src, workdir)),
    ]


@pytest.fixture(scope="module")
def printed(golden_dir):
    return (S._read_fields(os.path.join(golden_dir, "zipper_printed.txt")),
            S._read_fields(os.path.join(golden_dir, "permute_printed.txt")))


def test_unmutated_copy_passes_battery(tmp_path, printed):
    lib = oracle.compile_source(SRC, str(tmp_path / "liborig.so"))
    with oracle.using(lib):
        for check in _battery(*printed, SRC, tmp_path):
            check()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path, printed):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    mutated = src.replace(old, new)
    path = tmp_path / "mut.c"
    path.write_text(mutated)
    lib = oracle.compile_source(str(path), str(tmp_path / "libmut.so"))
    checks = ([S.test_remainder_follows_documented_reading] if name in UNPINNED
              else _battery(*printed, str(path), tmp_path))
    caught = []
    with oracle.using(lib):
        for i, check in enumerate(checks):
            try:
                check()
            except AssertionError:
                caught.append(i)
                break
    assert caught, "no pin caught: " + name


@pytest.mark.parametrize("name", sorted(UNPINNED))
def test_unpinned_reading_passes_the_paper_pins(name, tmp_path, printed):
    """The rotate direction is a convention: flipping it breaks no pin that
    the paper fixes (only the conformance test), which is why it is listed as
    parity unpinned."""
    old, new = MUTATIONS[name]
    src = open(SRC).read().replace(old, new)
    path = tmp_path / "mut.c"
    path.write_text(src)
    lib = oracle.compile_source(str(path), str(tmp_path / "libmut.so"))
    with oracle.using(lib):
        for check in _battery(*printed, str(path), tmp_path)[:-1]:
            check()
