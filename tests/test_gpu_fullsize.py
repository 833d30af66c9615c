"""Full-size pools, compared bit for bit with the oracle's accepted sets.

The oracle's accepted draws of these pools are stored under tests/golden/ by
``tests/golden/make_pool_fixture.py``, which calls only ``oracle/`` (the oracle takes minutes to
hours on them, too long for a test).  Bar: the accepted keys are identical; M within 1e-9
relative where the library reports its FP64 recomputation (flag 1) and 1e-4 relative for FP32
values.

  precision_n1000_d1000: n = d = 1000, AR(1) + Student-t covariates, 2e5 draws, q = 0.01
      (2000 kept); the split BF16, FP32 and fixed-point int8 forms; randomization-test counts
      equal the oracle's exactly.
  refresh_n64_d8: 17.3e6 draws whose keys cross 2^32, q = 1e-4 (1731 kept): long enough for the
      running acceptance bound of the streaming prefilter to be refreshed twice.
  stream_n1000_d1000: n = d = 1000, 1e8 draws, q = 1.2e-5 (1200 kept), the streaming
      workload the benchmark times, in the split BF16 and fixed-point int8 forms (and FP32).
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


DEV = "cuda:0"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def u64(t):
    return t.cpu().numpy().astype(np.uint64)


def fixture(name):
    path = os.path.join(GOLDEN, f"pool_{name}.json")
    with open(path) as f:
        fx = json.load(f)
    w = inputs.WORKLOADS[name]
    for key in ("n", "n1", "d", "seed", "key_begin", "num_draws", "q", "ridge_rel"):
        assert fx[key] == w[key], f"fixture {name} was written for another {key}"
    return fx, np.array(fx["keys"], dtype=np.uint64), np.array(fx["M"], dtype=np.float64)


def check_against_fixture(keys, M, flags, ref_keys, ref_M, label):
    got = u64(keys)
    assert len(got) == len(ref_keys), f"{label}: {len(got)} accepted, oracle {len(ref_keys)}"
    np.testing.assert_array_equal(got, ref_keys, err_msg=f"{label}: accepted keys differ from the oracle")
    Mg, fl = M.cpu().numpy(), flags.cpu().numpy().astype(bool)
    if fl.any():
        np.testing.assert_allclose(Mg[fl], ref_M[fl], rtol=1e-9)
    if (~fl).any():
        np.testing.assert_allclose(Mg[~fl], ref_M[~fl], rtol=1e-4)
    rel = np.abs(Mg[~fl] - ref_M[~fl]) / ref_M[~fl] if (~fl).any() else np.zeros(1)
    say(f"  {label}: {len(got)} keys identical; FP32 values max rel err {rel.max():.3e}; "
        f"FP64-reported {int(fl.sum())}")


def test_precision_pool_exact(rr):
    name = "precision_n1000_d1000"
    w = inputs.WORKLOADS[name]
    fx, ref_keys, ref_M = fixture(name)
    say("precision pool n=d=1000, 2e5 draws, against the oracle's accepted set")
    X = inputs.workload_X(name)
    P = rr.rr_prepare(dev(X), w["n1"], w["ridge_rel"])
    forms = [("split", rr.PREC_SPLIT_BF16), ("fp32", rr.PREC_FP32), ("i8", rr.PREC_FIXED_I8)]
    out = {}
    for label, prec in forms:
        ks, Ms, fs = rr.rr_draw_balance(P, w["seed"], w["key_begin"], w["num_draws"], rr.MODE_QUANTILE, w["q"],
                                        prec)
        check_against_fixture(ks, Ms, fs, ref_keys, ref_M, label)
        out[label] = ks
    # randomization test on the accepted pool
    obs = inputs.obs_pick(len(ref_keys), w["obs_seed"])
    wo = pipeline.regenerate(w["seed"], ref_keys[obs:obs + 1], w["n"], w["n1"])[0]
    Y = inputs.outcomes(X, wo, w["tau"], w["noise_sd"], w["y_seed"])
    taus = w["taus"][::10]
    counts, tau_hat = rr.rr_rand_test(P, w["seed"], out["split"], obs, dev(Y), taus)
    ref = pipeline.rand_test_keys(w["seed"], ref_keys, w["n"], w["n1"], obs, Y, taus)
    assert counts.cpu().tolist() == ref["counts"]
    assert abs(tau_hat - ref["tau_hat"]) <= 1e-12 * max(1.0, abs(ref["tau_hat"]))


def test_refresh_pool_exact(rr):
    name = "refresh_n64_d8"
    w = inputs.WORKLOADS[name]
    fx, ref_keys, ref_M = fixture(name)
    say(f"streaming pool n=64 d=8, {w['num_draws']} draws from key {w['key_begin']}, against the oracle")
    X = inputs.workload_X(name)
    P = rr.rr_prepare(dev(X), w["n1"], w["ridge_rel"])
    for label, prec in [("split", rr.PREC_SPLIT_BF16), ("fp32", rr.PREC_FP32), ("i8", rr.PREC_FIXED_I8)]:
        ks, Ms, fs = rr.rr_draw_balance(P, w["seed"], w["key_begin"], w["num_draws"], rr.MODE_QUANTILE, w["q"],
                                        prec)
        t = rr.rr_last_timing()
        say(f"  {label}: {t['launches']} chunks, band {t['band']}")
        assert t["launches"] > 16, "the pool must span more than 16 chunks (two bound refreshes)"
        check_against_fixture(ks, Ms, fs, ref_keys, ref_M, label)


def test_stream_pool_exact(rr):
    name = "stream_n1000_d1000"
    w = inputs.WORKLOADS[name]
    if not os.path.exists(os.path.join(GOLDEN, f"pool_{name}.json")):
        pytest.skip("oracle fixture of the 1e8-draw pool not written")
    fx, ref_keys, ref_M = fixture(name)
    say("stream pool n=d=1000, 1e8 draws, q=1.2e-5, against the oracle's accepted set")
    X = inputs.workload_X(name)
    P = rr.rr_prepare(dev(X), w["n1"], w["ridge_rel"])
    for label, prec in [("split", rr.PREC_SPLIT_BF16), ("i8", rr.PREC_FIXED_I8), ("fp32", rr.PREC_FP32)]:
        ks, Ms, fs = rr.rr_draw_balance(P, w["seed"], w["key_begin"], w["num_draws"], rr.MODE_QUANTILE, w["q"],
                                        prec)
        t = rr.rr_last_timing()
        say(f"  {label}: {t['total_ms']:.1f} ms, band {t['band']}")
        check_against_fixture(ks, Ms, fs, ref_keys, ref_M, label)
