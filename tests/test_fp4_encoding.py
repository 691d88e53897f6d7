"""The matrix-core scan's operand encoding, checked on the CPU.

The scan turns each 32-bit sketch word into four FP4 (E2M1) operands, one per
bit class d: class 0 keeps bit 0 of every nibble, class 1 bit 1, class 2 bit
2, and class 3 is the word shifted down three places, masked to bit 0. With
E8M0 block scales 2, 1, 1/2, 2 (exponents 128, 127, 126, 128) every product of
two set bits is exactly 1.0, so the sum over the four classes of the scaled
FP4 dot products of two words is |a AND b|. E2M1 is decoded here from its
definition (OCP Microscaling formats: sign bit 3, two exponent bits with bias
1, one mantissa bit; exponent 0 is subnormal, 0.5 times the mantissa).
"""
import numpy as np

MASKS = [(0, 0x11111111), (0, 0x22222222), (0, 0x44444444), (3, 0x11111111)]  # (shift, mask)
SCALE_EXP = [128, 127, 126, 128]


def e2m1(nibble: int) -> float:
    sign = -1.0 if nibble & 8 else 1.0
    e, m = (nibble >> 1) & 3, nibble & 1
    return sign * (0.5 * m if e == 0 else 2.0 ** (e - 1) * (1 + 0.5 * m))


def class_operand(word: int, d: int):
    shift, mask = MASKS[d]
    v = (word >> shift) & mask
    return [e2m1((v >> (4 * i)) & 15) for i in range(8)]


def scaled_dot(a: int, b: int) -> float:
    total = 0.0
    for d in range(4):
        s = 2.0 ** (SCALE_EXP[d] - 127)
        total += sum((x * s) * (y * s) for x, y in zip(class_operand(a, d), class_operand(b, d)))
    return total


def test_e2m1_values_used():
    assert [e2m1(n) for n in (0, 1, 2, 4)] == [0.0, 0.5, 1.0, 2.0]


def test_class_products_are_and_popcounts():
    rng = np.random.default_rng(1910)
    words = [0, 0xFFFFFFFF, 0x80000000, 0x00000001, 0x88888888, 0x77777777]
    words += [int(x) for x in rng.integers(0, 2**32, size=200, dtype=np.uint64)]
    for a, b in zip(words, words[::-1]):
        assert scaled_dot(a, b) == bin(a & b).count("1"), (hex(a), hex(b))


def test_classes_partition_the_bits():
    # every bit of a word lands in exactly one class operand, as 0.5, 1 or 2
    for bit in range(32):
        w = 1 << bit
        hits = [(d, i) for d in range(4) for i, v in enumerate(class_operand(w, d)) if v != 0.0]
        assert hits == [(bit % 4, bit // 4)]
