"""The bf16-piece form of an FP32 product that the matrix-core convolution and
correlation use by default (umbir_tuning.products = 2), checked as arithmetic
on the host: an FP32 value is the exact sum of three bf16 pieces (each the
remainder so far rounded to 8 significant bits, to nearest even), and the six
piece products a_i b_j with i + j <= 4 give a b within FP32 rounding.  This
pins the error statement the design relies on; the device's own results are
held to the FP64 oracle by the GPU parity tests."""
import numpy as np


def to_bf16(x):
    """x (float32) rounded to bf16, to nearest even, as float32."""
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def pieces(x):
    p1 = to_bf16(x)
    r1 = (x - p1).astype(np.float32)
    p2 = to_bf16(r1)
    r2 = (r1 - p2).astype(np.float32)
    p3 = to_bf16(r2)
    return p1, p2, p3, r2


def test_three_pieces_are_exact_and_small():
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(400_000) * np.exp(rng.uniform(-40, 40, 400_000))).astype(np.float32)
    p1, p2, p3, r2 = pieces(x)
    assert np.array_equal(p3, r2)  # the last remainder needs no rounding
    assert np.array_equal(p1.astype(np.float64) + p2 + p3, x.astype(np.float64))
    assert np.all(np.abs(p2) <= 2.0 ** -8 * np.abs(x))
    assert np.all(np.abs(p3) <= 2.0 ** -16 * np.abs(x))
    # every piece is a bf16 value (low 16 bits zero)
    for p in (p1, p2, p3):
        assert np.all((p.view(np.uint32) & 0xFFFF) == 0)


def test_six_piece_products_within_fp32_rounding():
    rng = np.random.default_rng(2)
    a = rng.standard_normal(400_000).astype(np.float32)
    b = (rng.standard_normal(400_000) * 1e-3).astype(np.float32)
    A = [p.astype(np.float64) for p in pieces(a)[:3]]
    B = [p.astype(np.float64) for p in pieces(b)[:3]]
    six = A[0] * B[0] + A[0] * B[1] + A[1] * B[0] + A[0] * B[2] + A[1] * B[1] + A[2] * B[0]
    exact = a.astype(np.float64) * b.astype(np.float64)
    rel = np.abs(six - exact) / np.abs(exact)
    assert rel.max() <= 2.0 ** -23  # the three dropped products
    # a piece product is exact in FP32: 8 x 8 significant bits
    for i in range(3):
        for j in range(3):
            prod = A[i] * B[j]
            assert np.array_equal(prod.astype(np.float32).astype(np.float64), prod)
    # a dot product of the pieces in FP32 stays at FP32 level against FP64
    n = 4096
    terms = [(A[0], B[2]), (A[1], B[1]), (A[2], B[0]), (A[0], B[1]), (A[1], B[0]), (A[0], B[0])]
    acc = np.zeros(1, np.float32)
    for ai, bj in terms:
        acc = (acc + np.sum((ai[:n] * bj[:n]).astype(np.float32), dtype=np.float32)).astype(np.float32)
    dot32 = float(acc[0])
    ref = float(np.dot(a[:n].astype(np.float64), b[:n].astype(np.float64)))
    scale = float(np.dot(np.abs(a[:n]).astype(np.float64), np.abs(b[:n]).astype(np.float64)))
    assert abs(dot32 - ref) <= 64 * 2.0 ** -24 * scale
