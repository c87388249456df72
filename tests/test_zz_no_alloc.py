"""dmimo_beamform_noalloc: the scratch of dmimo_beamform in the library's
static device array, called through the C ABI.

Its outputs must equal dmimo_beamform's (with a caller workspace) bit for bit:
both run the same kernels on the same inputs.  Two calls in a row, the second
with a smaller input, so that the second call runs over what the first left
in the shared array.  Shapes: the batched one-pass kernel (K <= 8), the
general kernel with its Gram in the array (K = 16, M = 300), the persistent
kernel of dmimo_beamform_batched (K = 16, M <= 256, no scratch), and the
wide path of one large deployment (K = 32, M = 1024), whose per-tile shares
live in the array.  A call whose scratch would exceed the array is refused
before any launch.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2304_12745_amd import workloads as WL  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2304_12745_amd import dmimo
    dmimo.lib()
    return dmimo


def _H(B, K, M, seed):
    rng = np.random.default_rng(seed)
    return torch.from_numpy(WL.complex_normal(rng, (B, K, M), np.complex64)).cuda()


def _same(a, b):
    torch.cuda.synchronize()
    for name in ("W", "p_ant", "l21", "sinr", "rsum", "info"):
        x, y = getattr(a, name), getattr(b, name)
        assert torch.equal(x, y), name


# (first call, second smaller call): precoder, precision, B, K, M
CASES = [
    (("zf", "f32", 1024, 16, 300), ("zf", "f32", 100, 12, 280)),
    (("zf", "f64", 64, 8, 64), ("zf", "f64", 7, 5, 37)),
    (("zf", "f16x3", 512, 16, 256), ("zf", "f16x3", 3, 9, 130)),
    (("zf", "f16x3", 256, 16, 300), ("zf", "f16x3", 5, 16, 257)),
    (("zf", "f32", 1, 32, 1024), ("zf", "f32", 1, 20, 700)),
    (("mr", "f32", 2, 32, 1024), ("mr", "f32", 1, 16, 513)),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_equals_workspace_call(D, first, second):
    for i, (pc, prec, B, K, M) in enumerate((first, second)):
        print(f"beamform_noalloc call {i}: {pc} {prec} B={B} K={K} M={M}", flush=True)
        H = _H(B, K, M, 1000 * i + B + K + M)
        if prec == "f64":
            H = H.to(torch.complex128)
        ref = D.beamform(H, pc, None, 1e-12, 1.0, prec)
        got = D.beamform_noalloc(H, pc, None, 1e-12, 1.0, prec)
        _same(got, ref)
        assert int(got.info.abs().sum()) == 0


def test_noalloc_refuses_scratch_beyond_the_array(D):
    B, K, M = 8192, 16, 300                        # FP32 ZF: 16 MiB of Gram > 8 MiB
    need = D.workspace_size(D.CALL_BEAMFORM_ZF, B, K, M, 0, "f32")
    assert need > D.NOALLOC_SCRATCH_BYTES
    H = torch.zeros((B, K, M), dtype=torch.complex64, device="cuda")
    with pytest.raises(D.DmimoError) as e:
        D.beamform_noalloc(H, "zf", None, 1e-12, 1.0, "f32")
    assert e.value.status == 4                     # DMIMO_E_WORKSPACE
    # the largest batch that fits runs
    B = D.NOALLOC_SCRATCH_BYTES // (K * K * 8)
    H = _H(B, K, M, 5)
    _same(D.beamform_noalloc(H, "zf", None, 1e-12, 1.0, "f32"),
          D.beamform(H, "zf", None, 1e-12, 1.0, "f32"))
    # K = 16, M = 256 runs on the persistent batched kernel: no scratch at any B
    assert D.workspace_size(D.CALL_BEAMFORM_ZF, 8192, K, 256, 0, "f32") == 0
