"""CPU pins of the split-BF16 ("BF16x3") arithmetic that the reduced-precision
path uses for its complex products, emulated here in NumPy independently of
the kernels: x = hi + lo with hi = bf16(x) rounded to nearest even and
lo = bf16(x - hi); a real product is hi_a hi_b + hi_a lo_b + lo_a hi_b.

Bound used below.  BF16 keeps 8 significant bits, so its unit roundoff is
u = 2^-8.  Then |x - hi| <= u|x|, and |x - hi - lo| <= u|x - hi| <= u^2|x|.
Dropping lo_a lo_b and the two representation errors cost at most
(3 u^2 + O(u^3)) |a||b| per term.  The products of BF16 values are exact
in FP32, so FP32 accumulation over n terms adds gamma_n = n 2^-24 / (1 - n 2^-24)
times the sum of |terms|.
"""
import numpy as np
import torch

U = 2.0 ** -8


def bf16_rne(x):
    """Round FP32 values to BF16 (round to nearest, ties to even), kept as FP32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def split(x):
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_rne(x)
    lo = bf16_rne(x - hi)  # x - hi is exact in FP32
    return hi, lo


def prod3(a, b, acc):
    """Real matrix product in the three-product split form, accumulated in `acc`."""
    ah, al = split(a)
    bh, bl = split(b)
    f = lambda x: x.astype(acc)
    return f(ah) @ f(bh) + f(ah) @ f(bl) + f(al) @ f(bh)


def cprod3(A, B, acc):
    """Complex product from four real split products (real and imaginary planes)."""
    Ar, Ai = A.real.astype(np.float32), A.imag.astype(np.float32)
    Br, Bi = B.real.astype(np.float32), B.imag.astype(np.float32)
    return prod3(Ar, Br, acc) - prod3(Ai, Bi, acc), prod3(Ar, Bi, acc) + prod3(Ai, Br, acc)


def _unitary(d, rng):
    H = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    H = (H + H.conj().T) / 2
    w, Q = np.linalg.eigh(H)
    return (Q * np.exp(-1j * 0.7 * w)) @ Q.conj().T


def test_rounding_matches_torch_bfloat16():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000), rng.uniform(-1e-3, 1e-3, 20000),
                        np.array([0.0, 1.0, -1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8])]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(bf16_rne(x), ref)
    # ties go to even: 1 + 2^-8 sits halfway between 1 and 1 + 2^-7
    assert bf16_rne(np.float32(1.0 + 2.0 ** -8)) == np.float32(1.0)
    assert bf16_rne(np.float32(1.0 + 3 * 2.0 ** -8)) == np.float32(1.0 + 2.0 ** -6)


def test_split_represents_x_to_sixteen_bits():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(100000).astype(np.float32)
    hi, lo = split(x)
    assert np.all(np.abs(x - hi) <= U * np.abs(x))
    r = np.abs(x.astype(np.float64) - hi - lo)
    assert np.all(r <= U * U * np.abs(x))
    # and no better than that by much: the representation keeps about 16 bits
    assert np.max(r / np.abs(x)) > U * U / 4


def test_complex_product_within_the_derived_bound():
    d = 64
    rng = np.random.default_rng(2)
    A, B = _unitary(d, rng), _unitary(d, rng)
    A32 = A.astype(np.complex64).astype(np.complex128)  # what the kernel reads
    B32 = B.astype(np.complex64).astype(np.complex128)
    exact = A32 @ B32
    mag_r = np.abs(A32.real) @ np.abs(B32.real) + np.abs(A32.imag) @ np.abs(B32.imag)
    mag_i = np.abs(A32.real) @ np.abs(B32.imag) + np.abs(A32.imag) @ np.abs(B32.real)
    rep = 3 * U * U * (1 + 2 * U)
    n = 6 * d  # terms in one real or imaginary entry: 2 products x 3 splits x d
    gamma = n * 2.0 ** -24 / (1 - n * 2.0 ** -24)
    # exact accumulation: only the split errors remain
    cr, ci = cprod3(A, B, np.float64)
    assert np.all(np.abs(cr - exact.real) <= rep * mag_r)
    assert np.all(np.abs(ci - exact.imag) <= rep * mag_i)
    # FP32 accumulation as on the matrix cores
    cr, ci = cprod3(A, B, np.float32)
    assert np.all(np.abs(cr - exact.real) <= (rep + gamma) * mag_r)
    assert np.all(np.abs(ci - exact.imag) <= (rep + gamma) * mag_i)


def test_error_is_of_order_u_squared():
    """The split product keeps about 16 bits: its error is a fixed fraction of
    u^2 times sum |a||b|, and more than ten times that of a plain FP32
    product, whose products are not rounded to 16 bits."""
    d = 64
    rng = np.random.default_rng(3)
    a = rng.standard_normal((d, d)).astype(np.float32)
    b = rng.standard_normal((d, d)).astype(np.float32)
    exact = a.astype(np.float64) @ b.astype(np.float64)
    e3 = np.abs(prod3(a, b, np.float64) - exact).max()
    e32 = np.abs((a @ b).astype(np.float64) - exact).max()
    scale = (np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64)).max()
    assert U * U / 64 * scale <= e3 <= 3 * U * U * scale
    assert e32 < e3 / 10
