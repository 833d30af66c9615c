"""rr_balance_keys_noalloc (the allocation-free variant) against rr_balance_keys (needs an MI355X).

Collected last on purpose: it must pass after every other test of the session as well as alone.

Two calls in a row on one handle, the second with fewer keys, each compared with
rr_balance_keys on the same keys: M32 and its bound bit for bit, M64 bit for bit (same
kernels); M64 also against the oracle on a sample.  Also: the size limit of the scratch array is
an error, not an overrun, and a handle of another shape reuses the same scratch correctly.
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import pipeline  # noqa: E402
from paper_2501_07642_amd import inputs  # noqa: E402


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


def run_noalloc(rr, P, seed, keys, prec):
    K = keys.numel()
    m32 = torch.empty(K, dtype=torch.float32, device="cuda:0")
    err = torch.empty(K, dtype=torch.float32, device="cuda:0")
    m64 = torch.empty(K, dtype=torch.float64, device="cuda:0")
    rr.rr_balance_keys_noalloc(P, seed, keys, m32, err, m64, prec)
    torch.cuda.synchronize()
    return m32, err, m64


@pytest.mark.parametrize("n,n1,d", [(1000, 500, 1000), (300, 120, 40)])
def test_noalloc_matches_balance_keys(rr, n, n1, d):
    say(f"noalloc n={n} d={d}")
    X = inputs.gaussian_X(n, d, 900 + n)
    P = rr.rr_prepare(torch.from_numpy(X).cuda(), n1, 1e-2)
    seed = 0x0A110C + n
    for K, prec in [(100_000, rr.PREC_SPLIT_BF16), (3_001, rr.PREC_SPLIT_BF16), (2_500, rr.PREC_FIXED_I8)]:
        keys = (torch.arange(K, dtype=torch.int64, device="cuda:0") * 104729 + 77) % (1 << 40)
        a32, aerr, a64 = run_noalloc(rr, P, seed, keys, prec)
        b32, berr, b64 = rr.rr_balance_keys(P, seed, keys, prec)
        assert torch.equal(a32, b32) and torch.equal(aerr, berr) and torch.equal(a64, b64), \
            f"K={K}: the allocation-free call differs from rr_balance_keys"
        s = keys[:: max(1, K // 40)].cpu().numpy().astype(np.uint64)
        ref = pipeline.balance_of_keys(X, n1, 1e-2, seed, s)
        np.testing.assert_allclose(a64[:: max(1, K // 40)].cpu().numpy(), ref, rtol=1e-9)
        say(f"  K={K}: identical to rr_balance_keys")


def test_noalloc_limit_and_m64_only(rr):
    X = inputs.gaussian_X(4096, 8, 991)
    P = rr.rr_prepare(torch.from_numpy(X).cuda(), 2048, 0.0)
    K = 131_072                      # one key above the limit at n = 4096 (S = 16: 512 B per key)
    keys = torch.arange(K, dtype=torch.int64, device="cuda:0")
    with pytest.raises(rr.RRError) as e:
        run_noalloc(rr, P, 5, keys, rr.PREC_SPLIT_BF16)
    assert e.value.status == "RR_E_UNSUPPORTED"
    # M64 alone needs no bitmask scratch
    m64 = torch.empty(K, dtype=torch.float64, device="cuda:0")
    rr.rr_balance_keys_noalloc(P, 5, keys, None, None, m64, rr.PREC_SPLIT_BF16)
    torch.cuda.synchronize()
    _, _, b64 = rr.rr_balance_keys(P, 5, keys[:1000], want_m32=False)
    assert torch.equal(m64[:1000], b64)
    # the largest accepted size works
    keys = keys[:131_071]
    a32, aerr, a64 = run_noalloc(rr, P, 5, keys, rr.PREC_SPLIT_BF16)
    b32, berr, _ = rr.rr_balance_keys(P, 5, keys, want_m64=False)
    assert torch.equal(a32, b32) and torch.equal(aerr, berr)
