"""HIP path vs the CPU oracle, through the C ABI (needs an MI355X).

Bar: assignments, accepted key sets and p-value counts bit-exact; M within 1e-9 relative
where the library reports its FP64 recomputation and 1e-4 relative for FP32 values; the
FP32 error bound must hold for every draw checked.
"""

import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import assign, balance, frt, pipeline, prep  # noqa: E402
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


DEV = "cuda:0"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


PRECS = {"split": lambda rr: rr.PREC_SPLIT_BF16, "fp32": lambda rr: rr.PREC_FP32,
         "i8": lambda rr: rr.PREC_FIXED_I8, "gram": lambda rr: rr.PREC_GRAM_BF16}


def u64(t):
    return t.cpu().numpy().astype(np.uint64)


def keys_t(keys):
    return dev(np.asarray(keys, dtype=np.uint64).astype(np.int64))


# one n per 256-unit chunk count 1..8 (the generators specialise on it) plus the largest n
@pytest.mark.parametrize("n,n1", [(2, 1), (5, 2), (20, 10), (64, 31), (100, 50), (257, 100), (600, 300),
                                  (1000, 500), (1100, 550), (1400, 699), (1700, 851), (2000, 1000),
                                  (4096, 2048)])
def test_regenerate_bits_exact(rr, n, n1):
    say(f"regenerate n={n} n1={n1}")
    X = inputs.gaussian_X(n, 3, 1)
    P = rr.rr_prepare(dev(X), n1, 1e-2)
    seed = 0xC0FFEE0000000000 + n
    keys = np.array([0, 1, 2, 77, 2 ** 32 - 1, 2 ** 32, 2 ** 40 + 3, 2 ** 64 - 1], dtype=np.uint64)
    got = rr.rr_regenerate(P, seed, keys_t(keys)).cpu().numpy().view(np.uint32)
    want = assign.pack_bits(assign.mc_assignments_batch(seed, keys, n, n1))
    np.testing.assert_array_equal(got, want)


def test_regenerate_exact_ranks(rr):
    n, n1 = 20, 10
    say("regenerate exact ranks")
    P = rr.rr_prepare(dev(inputs.gaussian_X(n, 3, 2)), n1, 0.0)
    ranks = np.array([0, 1, 2, 1000, 184755, 92377], dtype=np.uint64)
    got = rr.rr_regenerate(P, 0, keys_t(ranks), exact=True).cpu().numpy().view(np.uint32)
    want = assign.pack_bits(np.stack([assign.exact_assignment(int(r), n, n1) for r in ranks]))
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n,n1,d,ridge", [(20, 10, 3, 0.0), (60, 25, 8, 0.0), (100, 50, 100, 1e-2),
                                          (300, 150, 40, 0.0), (1000, 500, 1000, 1e-2), (96, 40, 300, 1.0)])
@pytest.mark.parametrize("prec", ["split", "fp32", "i8", "gram"])
def test_balance_values_and_bound(rr, n, n1, d, ridge, prec):
    say(f"balance n={n} d={d} prec={prec}")
    X = inputs.gaussian_X(n, d, 3)
    P = rr.rr_prepare(dev(X), n1, ridge)
    seed = 99
    keys = np.arange(5000, 5000 + 256, dtype=np.uint64)
    pr = PRECS[prec](rr)
    m32, err, m64 = rr.rr_balance_keys(P, seed, keys_t(keys), pr)
    m32, err, m64 = m32.cpu().numpy(), err.cpu().numpy(), m64.cpu().numpy()
    Pr = prep.prepare(X, n1, ridge)
    W = assign.mc_assignments_batch(seed, keys, n, n1)
    want = balance.mahalanobis_batch(X, W, Pr["S_lam"])
    np.testing.assert_allclose(m64, want, rtol=1e-9)
    if prec == "i8":
        # 15-bit fixed point: about 2^-13 sqrt(d / M) relative (the bound below is the contract)
        np.testing.assert_allclose(m32, want, rtol=5e-4 * np.sqrt(d / np.minimum(want, d)).max(), atol=1e-6 * d)
    elif prec == "gram":
        # w^T K w in FP32 can cancel; the bound below is the contract
        np.testing.assert_allclose(m32, want, rtol=1e-3, atol=1e-5 * d)
    else:
        np.testing.assert_allclose(m32, want, rtol=1e-4, atol=1e-4 * d * 1e-3)
    assert np.all(np.abs(m32.astype(np.float64) - m64) <= err)
    say(f"  max |m32-m64|/err = {np.max(np.abs(m32 - m64) / err):.3e}, err/M = {np.median(err / m64):.2e}")


def _check_pool(rr, X, n1, ridge, seed, N, mode, qa, prec):
    P = rr.rr_prepare(dev(X), n1, ridge)
    pr = PRECS[prec](rr)
    md = rr.MODE_QUANTILE if mode == "quantile" else rr.MODE_THRESHOLD
    keys, M, flags = rr.rr_draw_balance(P, seed, 0, N, md, qa, pr)
    acc, Macc, Mall = pipeline.draw_balance(X, n1, ridge, seed, 0, N, mode, qa)
    got = u64(keys)
    np.testing.assert_array_equal(got, acc)
    Mg, fl = M.cpu().numpy(), flags.cpu().numpy().astype(bool)
    np.testing.assert_allclose(Mg[fl], Macc[fl], rtol=1e-9)
    np.testing.assert_allclose(Mg[~fl], Macc[~fl], rtol=1e-4)
    if prec in ("i8", "gram"):
        assert fl.all()   # these forms report FP64 M for every accepted draw
    return P, got, rr.rr_last_timing()


@pytest.mark.parametrize("prec", ["split", "fp32", "i8", "gram"])
@pytest.mark.parametrize("mode,qa", [("quantile", 0.05), ("quantile", 1e-3), ("threshold", 4.0)])
def test_pool_small(rr, prec, mode, qa):
    say(f"pool small {mode} {qa} {prec}")
    X = inputs.gaussian_X(60, 8, 5)
    _, got, t = _check_pool(rr, X, 30, 0.0, 4242, 4000, mode, qa, prec)
    say(f"  accepted {len(got)} band {t['band']}")


@pytest.mark.parametrize("prec", ["split", "fp32", "i8", "gram"])
@pytest.mark.parametrize("mode,qa", [("quantile", 1.0), ("threshold", float("inf")), ("threshold", 0.0),
                                     ("threshold", -1.0)])
def test_pool_accept_all_or_none(rr, prec, mode, qa):
    """Degenerate acceptance: q = 1 and an infinite threshold keep every draw (in key order), a
    threshold at or below zero keeps none (M >= 0), as in the oracle."""
    say(f"pool accept all or none {mode} {qa} {prec}")
    X = inputs.gaussian_X(60, 8, 5)
    _, got, t = _check_pool(rr, X, 30, 0.0, 4242, 1500, mode, qa, prec)
    keep_all = mode == "quantile" or qa == float("inf")
    assert len(got) == (1500 if keep_all else 0)
    if keep_all:
        np.testing.assert_array_equal(got, np.arange(1500, dtype=np.uint64))
    say(f"  accepted {len(got)} band {t['band']}")


def test_pool_ragged_tiles(rr):
    # draw counts that leave partial tiles; n not a multiple of 16 / 32 / 64
    for n, d, N in [(37, 5, 1), (37, 5, 63), (101, 33, 129), (531, 70, 1000)]:
        say(f"pool ragged n={n} d={d} N={N}")
        X = inputs.gaussian_X(n, d, n)
        for prec in ("split", "i8"):
            _check_pool(rr, X, n // 3, 1e-3, 7, N, "quantile", 0.1, prec)


def test_exact_enumeration_c1(rr):
    w = inputs.WORKLOADS["exact_n20_d3"]
    say("exact enumeration n=20")
    X = inputs.workload_X("exact_n20_d3")
    P = rr.rr_prepare(dev(X), w["n1"], 0.0)
    for prec in (rr.PREC_SPLIT_BF16, rr.PREC_FP32, rr.PREC_FIXED_I8, rr.PREC_GRAM_BF16):
        keys, M, flags = rr.rr_draw_exact(P, rr.MODE_QUANTILE, w["q"], prec)
        acc, Macc, _ = pipeline.draw_exact(X, w["n1"], 0.0, "quantile", w["q"])
        assert len(acc) == 1848
        np.testing.assert_array_equal(u64(keys), acc)


def test_mc_c2_and_frt(rr):
    name = "mc_n100_d100"
    w = inputs.WORKLOADS[name]
    say("C2 pool + FRT")
    X = inputs.workload_X(name)
    P, acc, t = _check_pool(rr, X, w["n1"], w["ridge_rel"], w["seed"], w["num_draws"], "quantile", w["q"],
                            "fp32")
    assert len(acc) == 2000
    obs = inputs.obs_pick(len(acc), w["obs_seed"])
    wo = pipeline.regenerate(w["seed"], acc[obs:obs + 1], w["n"], w["n1"])[0]
    Y = inputs.outcomes(X, wo, w["tau"], w["noise_sd"], w["y_seed"])
    counts, tau_hat = rr.rr_rand_test(P, w["seed"], keys_t(acc), obs, dev(Y), w["taus"])
    ref = pipeline.rand_test_keys(w["seed"], acc, w["n"], w["n1"], obs, Y, w["taus"])
    assert counts.cpu().tolist() == ref["counts"]
    assert abs(tau_hat - ref["tau_hat"]) <= 1e-12 * max(1.0, abs(ref["tau_hat"]))
    assert min(ref["counts"]) >= 1


def test_rand_test_exact_c1(rr):
    name = "exact_n20_d3"
    w = inputs.WORKLOADS[name]
    say("C1 FRT")
    X = inputs.workload_X(name)
    P = rr.rr_prepare(dev(X), w["n1"], 0.0)
    keys, _, _ = rr.rr_draw_exact(P, rr.MODE_QUANTILE, w["q"], rr.PREC_SPLIT_BF16)
    acc = u64(keys)
    obs = inputs.obs_pick(len(acc), w["obs_seed"])
    wo = pipeline.regenerate(0, acc[obs:obs + 1], w["n"], w["n1"], exact=True)[0]
    Y = inputs.outcomes(X, wo, w["tau"], w["noise_sd"], w["y_seed"])
    counts, _ = rr.rr_rand_test(P, 0, keys, obs, dev(Y), w["taus"], exact=True)
    ref = pipeline.rand_test_keys(0, acc, w["n"], w["n1"], obs, Y, w["taus"], exact=True)
    assert counts.cpu().tolist() == ref["counts"]


def test_errors(rr):
    say("error paths")
    X = inputs.gaussian_X(10, 12, 1)
    with pytest.raises(rr.RRError) as e:
        rr.rr_prepare(dev(X), 5, 0.0)
    assert e.value.status == "RR_E_SINGULAR"
    P = rr.rr_prepare(dev(X), 5, 1e-2)
    with pytest.raises(rr.RRError) as e:
        rr.rr_draw_balance(P, 1, 0, 1000, rr.MODE_QUANTILE, 0.1, rr.PREC_SPLIT_BF16, capacity=50)
    assert e.value.status == "RR_E_CAPACITY" and e.value.count == 100
    keys, _, _ = rr.rr_draw_balance(P, 1, 0, 1000, rr.MODE_QUANTILE, 0.1, rr.PREC_SPLIT_BF16)
    with pytest.raises(rr.RRError) as e:
        rr.rr_rand_test(P, 1, keys, 100, dev(np.ones(10)), [0.0])
    assert e.value.status == "RR_E_OBS"
    with pytest.raises(rr.RRError) as e:
        rr.rr_rand_test(P, 1, keys, 0, dev(np.ones(10)), [1e-30])
    assert e.value.status == "RR_E_RANGE"
    P2 = rr.rr_prepare(dev(inputs.gaussian_X(70, 3, 1)), 35, 0.0)
    with pytest.raises(rr.RRError) as e:
        rr.rr_draw_exact(P2, rr.MODE_QUANTILE, 0.1, rr.PREC_SPLIT_BF16)
    assert e.value.status == "RR_E_RANGE"
    with pytest.raises(rr.RRError) as e:
        rr.rr_draw_balance(P, 1, 0, 1000, rr.MODE_QUANTILE, 0.0, rr.PREC_SPLIT_BF16)
    assert e.value.status == "RR_E_ARG"


@pytest.mark.parametrize("prec", ["split", "fp32", "i8", "gram"])
def test_diagonal_metric_pool(rr, prec):
    """Standardise-only metric: same kernels on the column-scaled covariates."""
    say(f"diagonal metric pool {prec}")
    rng = np.random.default_rng(77)
    X = rng.standard_normal((300, 40)) @ rng.standard_normal((40, 40)) * rng.uniform(0.1, 10.0, 40)
    pr = PRECS[prec](rr)
    P = rr.rr_prepare(dev(X), 120, 1e-3, metric=rr.METRIC_DIAGONAL)
    keys, M, flags = rr.rr_draw_balance(P, 99, 0, 20_000, rr.MODE_QUANTILE, 0.01, pr)
    acc, Macc, Mall = pipeline.draw_balance(X, 120, 1e-3, 99, 0, 20_000, "quantile", 0.01, metric="diagonal")
    np.testing.assert_array_equal(u64(keys), acc)
    Mg, fl = M.cpu().numpy(), flags.cpu().numpy().astype(bool)
    np.testing.assert_allclose(Mg[fl], Macc[fl], rtol=1e-9)
    np.testing.assert_allclose(Mg[~fl], Macc[~fl], rtol=1e-4)
    # the FP64 recheck path agrees with the oracle on arbitrary draws, and differs from the
    # whitened statistic on these correlated covariates
    ks = np.arange(0, 20_000, 97, dtype=np.uint64)
    _, _, m64 = rr.rr_balance_keys(P, 99, keys_t(ks), pr)
    np.testing.assert_allclose(m64.cpu().numpy(), Mall[ks.astype(np.int64)], rtol=1e-9)
    Mmah = pipeline.balance_of_keys(X, 120, 1e-3, 99, ks)
    assert np.max(np.abs(Mmah - Mall[ks.astype(np.int64)]) / Mmah) > 1e-2



@pytest.mark.parametrize("n,d,N", [(3000, 40, 3000), (4096, 24, 2048)])
def test_pool_large_n(rr, n, d, N):
    """n above 2048: 16 chunks of 256 units, generated with a runtime chunk count."""
    say(f"pool large n={n} d={d} N={N}")
    X = inputs.gaussian_X(n, d, n + 3)
    for prec in ("split", "fp32", "i8", "gram"):
        _check_pool(rr, X, n // 2 - 7, 1e-3, 99, N, "quantile", 0.02, prec)


@pytest.mark.parametrize("mode,qa", [("quantile", 0.003), ("threshold", 2.0)])
def test_exact_enumeration_unbalanced(rr, mode, qa):
    """All C(22, 6) = 74613 assignments of an unbalanced design (no M(w) = M(1 - w) pairs)."""
    say(f"exact n=22 n1=6 {mode}")
    X = inputs.gaussian_X(22, 4, 2201)
    P = rr.rr_prepare(dev(X), 6, 0.0)
    md = rr.MODE_QUANTILE if mode == "quantile" else rr.MODE_THRESHOLD
    for prec in (rr.PREC_SPLIT_BF16, rr.PREC_FP32, rr.PREC_FIXED_I8, rr.PREC_GRAM_BF16):
        keys, M, flags = rr.rr_draw_exact(P, md, qa, prec)
        acc, Macc, _ = pipeline.draw_exact(X, 6, 0.0, mode, qa)
        np.testing.assert_array_equal(u64(keys), acc)
        Mg, fl = M.cpu().numpy(), flags.cpu().numpy().astype(bool)
        np.testing.assert_allclose(Mg[fl], Macc[fl], rtol=1e-9)
        np.testing.assert_allclose(Mg[~fl], Macc[~fl], rtol=1e-4)


def test_chi2_threshold_mode(rr):
    """Acceptance at M <= c_q(d), the chi-square quantile (threshold from the approximation)."""
    from oracle import diagnose
    say("chi-square threshold mode")
    X = inputs.gaussian_X(100, 10, 31)
    P = rr.rr_prepare(dev(X), 40, 0.0)
    q, N = 0.05, 20_000
    a = diagnose.c_q(q, 10)
    for prec in (rr.PREC_SPLIT_BF16, rr.PREC_FP32, rr.PREC_FIXED_I8, rr.PREC_GRAM_BF16):
        keys, M, flags = rr.rr_draw_balance(P, 5, 0, N, rr.MODE_CHI2_QUANTILE, q, prec)
        acc, Macc, _ = pipeline.draw_balance(X, 40, 0.0, 5, 0, N, "threshold", a)
        np.testing.assert_array_equal(u64(keys), acc)
        np.testing.assert_allclose(M.cpu().numpy(), Macc, rtol=1e-9)
    assert abs(len(acc) / N - q) < 0.01      # M is close to chi^2_d here
    with pytest.raises(rr.RRError) as e:
        rr.rr_draw_balance(P, 5, 0, N, rr.MODE_CHI2_QUANTILE, 0.0, rr.PREC_SPLIT_BF16)
    assert e.value.status == "RR_E_ARG"


@pytest.mark.parametrize("prec", ["split", "gram"])
def test_high_dim_diagonal_pool(rr, prec):
    """d > n under the standardise-only metric, where the Gram form does n^2 work per draw."""
    say(f"high-dimensional diagonal pool n=200 d=768 {prec}")
    X = inputs.gaussian_X(200, 768, 4242)
    P = rr.rr_prepare(dev(X), 100, 0.0, metric=rr.METRIC_DIAGONAL)
    N = 20_000
    keys, M, flags = rr.rr_draw_balance(P, 8, 0, N, rr.MODE_QUANTILE, 0.01, PRECS[prec](rr))
    acc, Macc, _ = pipeline.draw_balance(X, 100, 0.0, 8, 0, N, "quantile", 0.01, metric="diagonal")
    np.testing.assert_array_equal(u64(keys), acc)
    Mg, fl = M.cpu().numpy(), flags.cpu().numpy().astype(bool)
    np.testing.assert_allclose(Mg[fl], Macc[fl], rtol=1e-9)
    np.testing.assert_allclose(Mg[~fl], Macc[~fl], rtol=1e-4)
    say(f"  accepted {len(acc)}, band {rr.rr_last_timing()['band']}")


@pytest.mark.parametrize("prec", ["split", "fp32", "i8", "gram"])
@pytest.mark.parametrize("n,d", [(60, 59), (60, 80)])
def test_pool_d_at_least_n_minus_1(rr, prec, n, d):
    """Whitened metric with d >= n - 1 (ridge 1e-3): M is nearly the same for every draw, so FP32
    cannot order the draws and most of them go through the FP64 guard band; the accepted set is
    still the oracle's."""
    say(f"pool d >= n - 1: n={n} d={d} {prec}")
    X = inputs.gaussian_X(n, d, 11 * d)
    _, got, t = _check_pool(rr, X, n // 2, 1e-3, 31, 5000, "quantile", 0.02, prec)
    say(f"  accepted {len(got)} band {t['band']}")


@pytest.mark.parametrize("prec", ["split", "fp32", "i8", "gram"])
def test_pool_extreme_n1(rr, prec):
    """One treated unit, and one control unit, in every operand form."""
    X = inputs.gaussian_X(97, 6, 977)
    for n1 in (1, 96):
        say(f"pool n=97 n1={n1} {prec}")
        _check_pool(rr, X, n1, 0.0, 31, 3000, "quantile", 0.02, prec)


@pytest.mark.parametrize("prec", ["split", "fp32", "i8", "gram"])
@pytest.mark.parametrize("n,d", [(50, 1), (500, 2), (257, 1)])
def test_pool_one_and_two_covariates(rr, prec, n, d):
    """d = 1 and 2: M is a single (or a sum of two) squared standardised difference(s); small
    values, one column block padded with 31 (or 30) zero columns."""
    say(f"pool n={n} d={d} {prec}")
    X = inputs.gaussian_X(n, d, 40 + n + d)
    _, got, t = _check_pool(rr, X, n // 2, 0.0, 777 + d, 30_000, "quantile", 0.004, prec)
    say(f"  accepted {len(got)} band {t['band']}")


def test_rand_test_interval_c2(rr):
    """Inversion of the test over the null grid: [min, max] of the grid values whose p-value
    exceeds alpha, and whether they are contiguous in the caller's grid order."""
    name = "mc_n100_d100"
    w = inputs.WORKLOADS[name]
    say("C2 fiducial interval")
    X = inputs.workload_X(name)
    P = rr.rr_prepare(dev(X), w["n1"], w["ridge_rel"])
    keys, _, _ = rr.rr_draw_balance(P, w["seed"], 0, 20_000, rr.MODE_QUANTILE, w["q"], rr.PREC_SPLIT_BF16)
    acc = u64(keys)
    obs = inputs.obs_pick(len(acc), w["obs_seed"])
    wo = pipeline.regenerate(w["seed"], acc[obs:obs + 1], w["n"], w["n1"])[0]
    Y = inputs.outcomes(X, wo, w["tau"], w["noise_sd"], w["y_seed"])
    taus = list(w["taus"])
    ref = pipeline.rand_test_keys(w["seed"], acc, w["n"], w["n1"], obs, Y, taus)
    K = len(acc)
    for alpha in (0.05, 0.2):
        counts, tau_hat, (lo, hi), contig = rr.rr_rand_test_interval(P, w["seed"], keys, obs, dev(Y), taus, alpha)
        assert counts.cpu().tolist() == ref["counts"]
        iv = frt.interval(taus, [c / K for c in ref["counts"]], alpha)
        assert (lo, hi, contig) == (iv["lo"], iv["hi"], iv["contiguous"]), (lo, hi, contig, iv)
        say(f"  alpha {alpha}: [{lo}, {hi}] contiguous {contig}, tau_hat {tau_hat:.3f}")
    # the same grid in a shuffled order: the kept values are no longer contiguous in that order
    perm = np.random.default_rng(3).permutation(len(taus))
    shuffled = [taus[i] for i in perm]
    counts, _, (lo, hi), contig = rr.rr_rand_test_interval(P, w["seed"], keys, obs, dev(Y), shuffled, 0.05)
    iv = frt.interval(shuffled, [ref["counts"][i] / K for i in perm], 0.05)
    assert (lo, hi, contig) == (iv["lo"], iv["hi"], iv["contiguous"]) and contig is False
    # no grid value kept: both ends NaN, reported contiguous
    far = [10.0, 11.0, -12.5]
    _, _, (lo, hi), contig = rr.rr_rand_test_interval(P, w["seed"], keys, obs, dev(Y), far, 0.05)
    assert math.isnan(lo) and math.isnan(hi) and contig
    with pytest.raises(rr.RRError):
        rr.rr_rand_test_interval(P, w["seed"], keys, obs, dev(Y), taus, 1.0)


def test_rand_test_range_edges(rr):
    """Null values at the edges of the always-accepted range (|tau0| = 2^-8, just below 2^20)
    and their negatives: counts equal the oracle's exact rational counts."""
    say("FRT range edges")
    X = inputs.gaussian_X(80, 5, 9)
    P = rr.rr_prepare(dev(X), 40, 0.0)
    keys, _, _ = rr.rr_draw_balance(P, 21, 0, 40_000, rr.MODE_QUANTILE, 0.01, rr.PREC_SPLIT_BF16)
    acc = u64(keys)
    wo = pipeline.regenerate(21, acc[7:8], 80, 40)[0]
    Y = inputs.outcomes(X, wo, 0.3, 1.0, 10)
    edge = math.nextafter(2.0 ** 20, 0.0)
    taus = [2.0 ** -8, -2.0 ** -8, math.nextafter(2.0 ** -8, 1.0), edge, -edge, 0.0, 1e5 + 0.125]
    counts, _ = rr.rr_rand_test(P, 21, keys, 7, dev(Y), taus)
    ref = pipeline.rand_test_keys(21, acc, 80, 40, 7, Y, taus)
    assert counts.cpu().tolist() == ref["counts"]
