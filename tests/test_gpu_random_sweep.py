"""Seeded random sweep through the C ABI: each case draws a method, a tile
variant (or a transposition of either operand), the three sizes, and for every
operand a padded leading dimension and an element offset into its allocation.
Padding holds NaN, so a kernel that touched an element outside its matrix
would show it.  Every result is checked against the oracle: the per-entry
bound of the sum for binary64 and FP32, the bfloat16 plane emulation for the
split methods, and bit equality on integer inputs for every method."""
import numpy as np
import pytest

import oracle
from paper_2408_15384_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

METHODS = ("f64", "f32", "split3", "split6")
CASES = 160


@pytest.fixture(scope="module")
def mm():
    from paper_2408_15384_amd import api
    api.load_library()
    assert api.lib().mm_init(0) == 0, api.lib().mm_last_error()
    return api


def stored(host, pad, off, dtype):
    """Device copy of a row-major host matrix with leading dimension
    cols + pad, starting `off` elements into a NaN-filled allocation."""
    r, c = host.shape
    ld = c + pad
    buf = torch.full((off + r * ld + 16,), float("nan"), dtype=dtype, device="cuda")
    view = buf.as_strided((r, c), (ld, 1), off)
    view.copy_(torch.from_numpy(np.ascontiguousarray(host)).to(dtype))
    return view, buf


def draw_case(i):
    rng = np.random.default_rng((2024, i))
    method = METHODS[i % 4]
    M, N, K = (int(x) for x in I.log_uniform_dims(rng, 3, 1, 700))
    integer = rng.random() < 0.25
    transposed = rng.random() < 0.3
    opa = "T" if transposed and rng.random() < 0.5 else "N"
    opb = "T" if transposed and (opa == "N" or rng.random() < 0.5) else "N"
    pads = [int(rng.integers(0, 8)) for _ in range(3)]
    offs = [int(rng.integers(0, 4)) for _ in range(3)]
    vpick = int(rng.integers(0, 1 << 30))
    return method, M, N, K, integer, opa, opb, pads, offs, vpick


@pytest.mark.parametrize("i", range(CASES))
def test_random_case(mm, i):
    method, M, N, K, integer, opa, opb, pads, offs, vpick = draw_case(i)
    f64 = method == "f64"
    kind = ("int_f64" if f64 else "int_f32") if integer else ("uniform_f64" if f64 else "uniform_f32")
    A, B = I.pair(kind, M, N, K, seed=(2025, i))
    dt = torch.float64 if f64 else torch.float32
    Ad, _ = stored(A.T if opa == "T" else A, pads[0], offs[0], dt)
    Bd, _ = stored(B.T if opb == "T" else B, pads[1], offs[1], dt)
    Cd, Cbuf = stored(np.zeros((M, N)), pads[2], offs[2], dt)
    Cd.fill_(float("nan"))
    if opa == "N" and opb == "N":
        variant = vpick % mm.variant_count(method)
        mm.gemm_variant(method, variant, Ad, Bd, Cd)
        label = f"{method} v{variant}"
    else:
        mm.gemm_ex(method, Ad, Bd, opa, opb, C=Cd)
        label = f"{method} {opa}{opb}"
    torch.cuda.synchronize()
    C = Cd.cpu().numpy()
    case = f"case {i}: {label} M={M} N={N} K={K} pads={pads} offs={offs} integer={integer}"
    # C's padding and the rest of its allocation are untouched
    whole = Cbuf.cpu().numpy()
    mask = np.ones(whole.shape, bool)
    ld = N + pads[2]
    for r in range(M):
        mask[offs[2] + r * ld: offs[2] + r * ld + N] = False
    assert np.all(np.isnan(whole[mask])), case + ": wrote outside C"
    if integer:
        R = oracle.gemm(A, B)
        assert np.array_equal(C.astype(np.float64), R), case
        return
    if method in ("split3", "split6"):
        R = oracle.split_product(A, B, int(method[-1]))
        bound = oracle.elementwise_bound(oracle.abs_product(A, B), K, oracle.U_F32) + 2.0 ** -24 * np.abs(R)
    else:
        R = oracle.gemm(A, B)
        bound = oracle.elementwise_bound(oracle.abs_product(A, B), K, oracle.U_F64 if f64 else oracle.U_F32)
    assert np.all(np.isfinite(C)), case + ": non-finite result"
    assert np.all(np.abs(C.astype(np.float64) - R) <= bound), case


GROUPED_CASES = 32


def pair_member(mm, method, variant, M, N, K):
    """The tile variant a grouped variant id runs an M x N x K problem on: the
    id itself, or for a size-class pair its small member when that member's
    tiles execute at most pct % of the large one's padded work, else its large
    member."""
    if variant < mm.PAIR_BASE:
        return variant
    small, large, pct = mm.grouped_pair_info(method, variant - mm.PAIR_BASE)

    def work(v):
        bm, bn, bk = mm.variant_info(method, v)
        return -(-M // bm) * bm * (-(-N // bn) * bn) * (-(-max(K, 1) // bk) * bk)
    return small if work(small) * 100 <= pct * work(large) else large


@pytest.mark.parametrize("i", range(GROUPED_CASES))
def test_random_grouped(mm, i):
    """A random batch (1-40 problems, sizes 1-300, padded and offset operands)
    under a random variant and schedule: each result equals the single-problem
    kernel of that variant bit for bit, stays within the oracle bound, and
    nothing outside the C matrices is written."""
    rng = np.random.default_rng((2026, i))
    method = METHODS[i % 4]
    # a tile variant or a size-class pair (grouped ids PAIR_BASE + p)
    nv = mm.variant_count(method)
    variant = int(rng.integers(0, nv + mm.grouped_pair_count(method)))
    if variant >= nv:
        variant = mm.PAIR_BASE + variant - nv
    schedule = int(rng.integers(0, 4))
    count = int(rng.integers(1, 41))
    f64 = method == "f64"
    dt = torch.float64 if f64 else torch.float32
    As, Bs, Cs, Cbufs, host, lay = [], [], [], [], [], []
    for j in range(count):
        M, N, K = (int(x) for x in I.log_uniform_dims(rng, 3, 1, 300))
        A, B = I.pair("uniform_f64" if f64 else "uniform_f32", M, N, K, seed=(2027, i, j))
        pads = [int(rng.integers(0, 8)) for _ in range(3)]
        offs = [int(rng.integers(0, 4)) for _ in range(3)]
        Ad, _ = stored(A, pads[0], offs[0], dt)
        Bd, _ = stored(B, pads[1], offs[1], dt)
        Cd, Cbuf = stored(np.zeros((M, N)), pads[2], offs[2], dt)
        Cd.fill_(float("nan"))
        As.append(Ad), Bs.append(Bd), Cs.append(Cd), Cbufs.append(Cbuf), host.append((A, B)), lay.append((pads, offs))
    mm.gemm_grouped(method, As, Bs, Cs, variant=variant, schedule=schedule)
    torch.cuda.synchronize()
    for j in range(count):
        A, B = host[j]
        M, K = A.shape
        N = B.shape[1]
        pads, offs = lay[j]
        case = f"case {i}: {method} v{variant} s{schedule} problem {j}/{count} M={M} N={N} K={K} pads={pads} offs={offs}"
        ref = torch.full((M, N), float("nan"), dtype=dt, device="cuda")
        mm.gemm_variant(method, pair_member(mm, method, variant, M, N, K), As[j], Bs[j], ref)
        torch.cuda.synchronize()
        C = Cs[j].cpu().numpy()
        assert np.array_equal(C, ref.cpu().numpy()), case + ": differs from the single-problem kernel"
        whole = Cbufs[j].cpu().numpy()
        mask = np.ones(whole.shape, bool)
        ld = N + pads[2]
        for r in range(M):
            mask[offs[2] + r * ld: offs[2] + r * ld + N] = False
        assert np.all(np.isnan(whole[mask])), case + ": wrote outside C"
        if method in ("split3", "split6"):
            R = oracle.split_product(A, B, int(method[-1]))
            bound = oracle.elementwise_bound(oracle.abs_product(A, B), K, oracle.U_F32) + 2.0 ** -24 * np.abs(R)
        else:
            R = oracle.gemm(A, B)
            bound = oracle.elementwise_bound(oracle.abs_product(A, B), K, oracle.U_F64 if f64 else oracle.U_F32)
        assert np.all(np.abs(C.astype(np.float64) - R) <= bound), case
