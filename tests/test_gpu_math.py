"""The vertex programs' rounded arithmetic on the GPU through the C ABI.

The normative FP32 programs need correctly rounded division and square root.
The library's reciprocal, square root and reciprocal square root (both
operations rounded) must equal the compiler's IEEE sequences on every one of
the 2^32 float32 operands, and numpy's IEEE-754 float32 results on the host
over ranges that cover the fast paths' edges, denormals, huge values,
negatives, infinities and NaNs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def stage():
    from paper_1805_08893_amd import vr
    s = vr.GeometryStage(0)
    yield s
    s.close()


def _bits(x):
    return int(np.array([x], dtype=np.float32).view(np.uint32)[0])


@pytest.mark.parametrize("fn", [0, 1, 2], ids=["recip", "sqrt", "recip_sqrt"])
def test_every_float32_operand(stage, fn):
    from paper_1805_08893_amd import vr
    st, bad = vr.vr_math_selftest(stage.ctx, fn)
    assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
    assert bad == 0


RANGES = {
    "around_one": (_bits(1.0) - (1 << 19), 1 << 20),
    "recip_low_edge": (_bits(2.0 ** -125) - (1 << 16), 1 << 17),
    "recip_high_edge": (_bits(2.0 ** 125) - (1 << 16), 1 << 17),
    "sqrt_low_edge": (_bits(2.0 ** -96) - (1 << 16), 1 << 17),
    "sqrt_high_edge": (_bits(2.0 ** 126) - (1 << 16), 1 << 17),
    "zero_and_denormals": (0, 1 << 20),
    "huge_inf_nan": (0x7F700000, 0x80000000 - 0x7F700000),
    "negative": (_bits(-1.0) - (1 << 19), 1 << 20),
    "negative_zero_denormals": (0x80000000, 1 << 20),
}


def _host(fn, x):
    with np.errstate(all="ignore"):
        if fn == 0:
            return np.float32(1) / x
        if fn == 1:
            return np.sqrt(x)
        return np.float32(1) / np.sqrt(x)


@pytest.mark.parametrize("name", sorted(RANGES))
@pytest.mark.parametrize("fn", [0, 1, 2], ids=["recip", "sqrt", "recip_sqrt"])
def test_against_host_ieee(stage, fn, name):
    from paper_1805_08893_amd import vr
    first, count = RANGES[name]
    out = torch.empty(count, dtype=torch.float32, device="cuda")
    st, bad = vr.vr_math_selftest(stage.ctx, fn, first, count, out)
    assert st == vr.VR_OK, vr.vr_last_error(stage.ctx)
    assert bad == 0
    got = out.cpu().numpy()
    x = np.arange(first, first + count, dtype=np.uint64).astype(np.uint32).view(np.float32)
    want = _host(fn, x).astype(np.float32)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan].view(np.uint32), want[~nan].view(np.uint32))


def test_argument_rules(stage):
    from paper_1805_08893_amd import vr
    assert vr.vr_math_selftest(stage.ctx, 3, 0, 1)[0] == vr.VR_ERR_ARG
    assert vr.vr_math_selftest(stage.ctx, 0, 1 << 32, 1)[0] == vr.VR_ERR_ARG
    assert vr.vr_math_selftest(stage.ctx, 0, (1 << 32) - 1, 2)[0] == vr.VR_ERR_ARG
    assert vr.vr_math_selftest(stage.ctx, 0, (1 << 32) - 1, 1)[0] == vr.VR_OK   # the last operand
    assert vr.vr_math_selftest(stage.ctx, 1, 0, 0)[0] == vr.VR_OK               # empty range
