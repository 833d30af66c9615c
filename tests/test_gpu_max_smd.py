"""Per-column criterion (largest squared standardised mean difference) on the GPU against the
oracle (needs an MI355X).

M_max(w) = (n1 n0 / n) max_j Delta_j^2 / (S_jj + lambda): the contraction keeps the largest
G_j^2 instead of the sum, the guard band uses the largest column bound, and the FP64 recheck
takes the maximum too.  Bar: accepted keys bit-exact, M within 1e-9 (FP64-reported) or 1e-4.
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def u64(t):
    return t.cpu().numpy().astype(np.uint64)


PRECS = {"split": "PREC_SPLIT_BF16", "fp32": "PREC_FP32", "i8": "PREC_FIXED_I8"}


def check(keys, M, flags, acc, Macc, label):
    np.testing.assert_array_equal(u64(keys), acc, err_msg=f"{label}: accepted keys differ")
    Mg, fl = M.cpu().numpy(), flags.cpu().numpy().astype(bool)
    if fl.any():
        np.testing.assert_allclose(Mg[fl], Macc[fl], rtol=1e-9)
    if (~fl).any():
        np.testing.assert_allclose(Mg[~fl], Macc[~fl], rtol=1e-4)


@pytest.mark.parametrize("prec", ["split", "fp32", "i8"])
@pytest.mark.parametrize("n,n1,d,N,mode,qa", [(300, 120, 40, 20_000, "quantile", 0.01),
                                             (1000, 500, 200, 30_000, "quantile", 0.003),
                                             (97, 48, 7, 25_001, "threshold", 0.5),
                                             (2500, 1250, 70, 8_000, "quantile", 0.02)])
def test_max_smd_pool(rr, prec, n, n1, d, N, mode, qa):
    say(f"max-SMD pool n={n} d={d} N={N} {mode} {qa} {prec}")
    rng = np.random.default_rng(n + d)
    X = rng.standard_normal((n, d)) @ rng.standard_normal((d, d)) * rng.uniform(0.1, 10.0, d)
    P = rr.rr_prepare(dev(X), n1, 1e-3, metric=rr.METRIC_MAX_SMD)
    m = rr.MODE_QUANTILE if mode == "quantile" else rr.MODE_THRESHOLD
    keys, M, flags = rr.rr_draw_balance(P, 4242, 0, N, m, qa, getattr(rr, PRECS[prec]))
    acc, Macc, Mall = pipeline.draw_balance(X, n1, 1e-3, 4242, 0, N, mode, qa, metric="max_smd")
    check(keys, M, flags, acc, Macc, prec)
    say(f"  {len(acc)} accepted, band {rr.rr_last_timing()['band']}")
    # every draw's FP32 value within its bound of the FP64 one, which matches the oracle
    ks = np.arange(0, N, 37, dtype=np.uint64)
    m32, err, m64 = rr.rr_balance_keys(P, 4242, dev(ks.astype(np.int64)), getattr(rr, PRECS[prec]))
    m32, err, m64 = (t.cpu().numpy().astype(np.float64) for t in (m32, err, m64))
    np.testing.assert_allclose(m64, Mall[ks.astype(np.int64)], rtol=1e-9)
    assert np.all(np.abs(m32 - m64) <= err)


def test_max_smd_differs_from_sum_and_rejects_gram(rr):
    X = inputs.gaussian_X(200, 30, 5)
    P = rr.rr_prepare(dev(X), 100, 0.0, metric=rr.METRIC_MAX_SMD)
    Q = rr.rr_prepare(dev(X), 100, 0.0, metric=rr.METRIC_DIAGONAL)
    ks = dev(np.arange(500, dtype=np.int64))
    _, _, a = rr.rr_balance_keys(P, 3, ks)
    _, _, b = rr.rr_balance_keys(Q, 3, ks)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.all(a <= b * (1 + 1e-12)) and np.all(b <= 30 * a * (1 + 1e-12))
    with pytest.raises(rr.RRError) as e:
        rr.rr_draw_balance(P, 3, 0, 1000, rr.MODE_QUANTILE, 0.01, rr.PREC_GRAM_BF16)
    assert e.value.status == "RR_E_ARG"


def test_max_smd_batched(rr):
    shapes = [(150, 75, 12), (700, 350, 90), (64, 31, 5)]
    Ps, Xs, seeds = [], [], []
    for p, (n, n1, d) in enumerate(shapes):
        X = inputs.gaussian_X(n, d, 8000 + p)
        Xs.append(X)
        Ps.append(rr.rr_prepare(dev(X), n1, 1e-2, metric=rr.METRIC_MAX_SMD))
        seeds.append(777 + p)
    out = rr.rr_draw_balance_batched(Ps, seeds, 0, 12_000, rr.MODE_QUANTILE, 0.01, rr.PREC_SPLIT_BF16)
    for p, (n, n1, d) in enumerate(shapes):
        acc, Macc, _ = pipeline.draw_balance(Xs[p], n1, 1e-2, seeds[p], 0, 12_000, "quantile", 0.01,
                                             metric="max_smd")
        np.testing.assert_array_equal(u64(out[p][0]), acc)
        np.testing.assert_allclose(out[p][1].cpu().numpy(), Macc, rtol=1e-4)
