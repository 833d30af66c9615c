"""rr_draw_balance_async: the stream-ordered call against the synchronous one (needs an MI355X).

The asynchronous call enqueues everything and writes its count and status on the device;
its results must equal rr_draw_balance's bit for bit (keys, M, flags), device-detected errors
must leave the outputs untouched, and successive calls on one stream must stay ordered.
"""

import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import pipeline  # noqa: E402
from paper_2501_07642_amd import inputs  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2501_07642_amd as rr
    rr.load()
    return rr


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


PRECS = ["PREC_SPLIT_BF16", "PREC_FP32", "PREC_FIXED_I8", "PREC_GRAM_BF16"]


def same(sync_out, async_out):
    ks, Ms, fs = sync_out
    ka, Ma, fa, cnt, st = async_out
    K = int(cnt.item())
    assert int(st.item()) == 0 and K == ks.numel()
    assert torch.equal(ka[:K], ks) and torch.equal(Ma[:K], Ms) and torch.equal(fa[:K], fs)


@pytest.mark.parametrize("prec", PRECS)
def test_async_equals_sync(rr, prec):
    say(f"async vs sync {prec}")
    X = inputs.gaussian_X(300, 40, 61)
    P = rr.rr_prepare(dev(X), 120, 1e-2)
    pr = getattr(rr, prec)
    for mode, qa, N in [(rr.MODE_QUANTILE, 0.01, 300_000), (rr.MODE_THRESHOLD, 22.0, 150_000),
                        (rr.MODE_CHI2_QUANTILE, 0.02, 90_001)]:
        sync_out = rr.rr_draw_balance(P, 5150, 77, N, mode, qa, pr)
        async_out = rr.rr_draw_balance_async(P, 5150, 77, N, mode, qa, pr)
        torch.cuda.synchronize()
        same(sync_out, async_out)
        say(f"  mode {mode}: {sync_out[0].numel()} accepted, identical")


def test_async_capacity_on_device(rr):
    """Threshold mode with too small a capacity: RR_E_CAPACITY and the required count on the
    device, outputs untouched; a quantile count above the capacity is refused on the host."""
    X = inputs.gaussian_X(200, 10, 62)
    P = rr.rr_prepare(dev(X), 100, 0.0)
    ks, _, _ = rr.rr_draw_balance(P, 9, 0, 50_000, rr.MODE_THRESHOLD, 6.0, rr.PREC_SPLIT_BF16)
    need = ks.numel()
    assert need > 20
    cap = need - 7
    keys = torch.full((cap,), -5, dtype=torch.int64, device="cuda:0")
    M = torch.full((cap,), -1.0, dtype=torch.float64, device="cuda:0")
    flags = torch.full((cap,), 7, dtype=torch.uint8, device="cuda:0")
    _, _, _, cnt, st = rr.rr_draw_balance_async(P, 9, 0, 50_000, rr.MODE_THRESHOLD, 6.0, rr.PREC_SPLIT_BF16,
                                                capacity=cap, out=(keys, M, flags))
    torch.cuda.synchronize()
    assert rr._lib.STATUS[int(st.item())] == "RR_E_CAPACITY" and int(cnt.item()) == need
    assert bool((keys == -5).all()) and bool((M == -1.0).all()) and bool((flags == 7).all())
    with pytest.raises(rr.RRError) as e:
        rr.rr_draw_balance_async(P, 9, 0, 50_000, rr.MODE_QUANTILE, 0.01, rr.PREC_SPLIT_BF16, capacity=10)
    assert e.value.status == "RR_E_CAPACITY"


def test_async_calls_in_flight_and_side_stream(rr):
    """Three calls enqueued back to back on one handle and a non-default stream, then one wait."""
    X = inputs.gaussian_X(500, 60, 63)
    P = rr.rr_prepare(dev(X), 250, 1e-2)
    refs = [rr.rr_draw_balance(P, s, 0, 200_000, rr.MODE_QUANTILE, 0.005, rr.PREC_SPLIT_BF16) for s in (1, 2, 3)]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        outs = [rr.rr_draw_balance_async(P, s, 0, 200_000, rr.MODE_QUANTILE, 0.005, rr.PREC_SPLIT_BF16)
                for s in (1, 2, 3)]
    side.synchronize()
    for ref, out in zip(refs, outs):
        same(ref, out)


def test_async_streaming_refresh_pool(rr):
    """The 17.3e6-draw streaming pool (keys crossing 2^32, two refreshes of the running bound)
    against the oracle's accepted set."""
    name = "refresh_n64_d8"
    w = inputs.WORKLOADS[name]
    with open(os.path.join(GOLDEN, f"pool_{name}.json")) as f:
        fx = json.load(f)
    X = inputs.workload_X(name)
    P = rr.rr_prepare(dev(X), w["n1"], w["ridge_rel"])
    keys, M, flags, cnt, st = rr.rr_draw_balance_async(P, w["seed"], w["key_begin"], w["num_draws"],
                                                       rr.MODE_QUANTILE, w["q"], rr.PREC_SPLIT_BF16)
    torch.cuda.synchronize()
    K = int(cnt.item())
    assert int(st.item()) == 0 and K == fx["k"]
    np.testing.assert_array_equal(keys[:K].cpu().numpy().astype(np.uint64), np.array(fx["keys"], dtype=np.uint64))
    np.testing.assert_allclose(M[:K].cpu().numpy(), np.array(fx["M"]), rtol=1e-9)
