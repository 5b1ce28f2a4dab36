"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars:
- exact-arithmetic inputs (integer weights, W/N integral): tables, partition,
  prefix sums and splits equal the oracle's bit for bit;
- general inputs: partition and split positions equal the oracle's, aliases
  equal, probabilities within 2 ulp, and every item's reconstructed mass
  within 1e-12 relative of n*w_i/W (the oracle's dd checker);
- samples drawn from an identical table equal the oracle's bit for bit;
- chi-squared at 10^8 draws.
Paper: arXiv 2106.12270 (Sec. 2.2, Sec. 4, Sec. 5).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_2106_12270_amd as pkg
from paper_2106_12270_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pkg.lib()
    oracle.lib()
    yield
    torch.cuda.synchronize()


def gpu_build(w, chunk=None, split="binary", model=None):
    b = pkg.Builder(len(w), chunk, split, model, device=DEV)
    wd = torch.from_numpy(np.ascontiguousarray(w)).to(DEV)
    prob, alias = b.build(wd)
    torch.cuda.synchronize()
    st = int(b.status.item())
    return b, st, prob.cpu().numpy(), alias.cpu().numpy().view(np.uint32)


def to_rows(p, a):
    """A table as 16-byte device rows {prob, alias, 0}."""
    r = torch.zeros((len(p), 4), dtype=torch.int32, device=DEV)
    r.view(torch.float64)[:, 0] = torch.from_numpy(p).to(DEV)
    r[:, 2] = torch.from_numpy(a.view(np.int32)).to(DEV)
    return r


def ulp_diff(a, b):
    ai = a.view(np.int64)
    bi = b.view(np.int64)
    return np.abs(ai - bi)


# --------------------------------------------------------------------------
# exact-arithmetic inputs: bitwise
# --------------------------------------------------------------------------
EXACT_SIZES = [1, 2, 3, 63, 64, 65, 1000, 4095, 4096, 4097, 3 * 4096 + 77, 65537, (1 << 20) + 13]


@pytest.mark.parametrize("n", EXACT_SIZES)
@pytest.mark.parametrize("chunk", [64, 1024, 2048])
def test_exact_inputs_bitwise(n, chunk):
    w = inputs.exact_integers(n, seed=n * 7 + chunk, zero_frac=0.05)
    say("exact", n, chunk)
    b, st, p, a = gpu_build(w, chunk)
    assert st == pkg.ALIAS_OK
    op, oa, info = oracle.psa_build(w, chunk=chunk, with_splits=True)
    assert np.array_equal(a, oa)
    assert np.array_equal(p, op)
    it = b.intermediates()
    assert it["L"] == info["L"] and it["H"] == info["H"]
    assert np.array_equal(it["split_i"], info["split_i"].astype(np.uint32))
    assert np.array_equal(it["split_j"], info["split_j"].astype(np.uint32))
    sp = it["spill"]
    assert np.array_equal(sp[:, 0] + sp[:, 1], info["spill_hi"] + info["spill_lo"])


def test_exact_inputs_partition_and_prefix_bitwise():
    n = 3 * 4096 + 1001
    w = inputs.exact_integers(n, seed=5, max_w=1000, zero_frac=0.1)
    say("exact partition", n)
    b, st, p, a = gpu_build(w, 256)
    it = b.intermediates()
    tot = oracle.total(w)
    l_idx, l_w, h_idx, h_w = oracle.partition(w, tot[2:])
    assert np.array_equal(it["l_idx"], l_idx) and np.array_equal(it["h_idx"], h_idx)
    assert np.array_equal(it["l_w"], l_w) and np.array_equal(it["h_w"], h_w)
    hdr = it["header"]
    assert hdr.avg_hi + hdr.avg_lo == tot[2] + tot[3]
    slh, sll = oracle.prefix(l_w)
    shh, shl = oracle.prefix(h_w)
    for agg, (hi, lo), cnt in ((it["agg_l"], (slh, sll), len(l_w)), (it["agg_h"], (shh, shl), len(h_w))):
        q = np.arange(0, cnt + 1, 64)
        assert np.array_equal(agg[: len(q), 0] + agg[: len(q), 1], hi[q] + lo[q])


# --------------------------------------------------------------------------
# general inputs: partition/splits/aliases equal, probs within 2 ulp, invariant
# --------------------------------------------------------------------------
GENERAL = {
    "uniform": lambda n: inputs.uniform01(n, 11),
    "powerlaw": lambda n: inputs.power_law(n, 1.0, 11),
    "powerlaw_a05": lambda n: inputs.power_law(n, 0.5, 11),
    "lognormal": lambda n: inputs.lognormal(n, 2.0, 11),
    "lognormal_sorted_desc": lambda n: inputs.sorted_descending(inputs.lognormal(n, 2.0, 11)),
    "sorted_ascending": lambda n: np.sort(inputs.lognormal(n, 1.0, 11)),
    "one_heavy": lambda n: np.concatenate([[float(n)], np.ones(n - 1)]),
}


@pytest.mark.parametrize("name", list(GENERAL))
@pytest.mark.parametrize("n", [(1 << 18) + 77, 5000])
def test_general_inputs(name, n):
    w = GENERAL[name](n)
    say("general", name, n)
    b, st, p, a = gpu_build(w, 1024)
    assert st == pkg.ALIAS_OK
    op, oa, info = oracle.psa_build(w, chunk=1024, with_splits=True)
    it = b.intermediates()
    assert it["L"] == info["L"] and it["H"] == info["H"]
    assert np.array_equal(it["split_i"], info["split_i"].astype(np.uint32))
    assert np.array_equal(it["split_j"], info["split_j"].astype(np.uint32))
    assert np.array_equal(a, oa)
    assert ulp_diff(p, op).max() <= 2
    r = oracle.check(w, p, a)
    assert r["max_rel"] <= 1e-12, r
    assert r["sum_dev"] <= 1e-12
    assert r["zero_violations"] == 0


@pytest.mark.parametrize("name", ["powerlaw", "lognormal", "uniform"])
@pytest.mark.parametrize("n", [(1 << 18) + 77, 4097, 1])
def test_row_layout_equals_two_array_layout(name, n):
    w = GENERAL[name](n) if n > 1 else np.array([2.5])
    say("rows", name, n)
    b, st, p, a = gpu_build(w, 1024)
    rows = b.build_rows(torch.from_numpy(w).to(DEV))
    torch.cuda.synchronize()
    assert int(b.status.item()) == 0
    r = rows.cpu().numpy()
    assert np.array_equal(r[:, :2].copy().view(np.float64).ravel(), p)
    assert np.array_equal(r[:, 2].view(np.uint32), a)
    assert np.all(r[:, 3] == 0)
    # the same draws from both layouts of the GPU table
    pd = torch.from_numpy(p).to(DEV)
    ad = torch.from_numpy(a.view(np.int32)).to(DEV)
    o1 = pkg.sample(pd, ad, 300_001, 77, first_draw=12345)
    o2 = pkg.sample_rows(rows, 300_001, 77, first_draw=12345)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)
    # both layouts of the oracle's table: draws equal to the oracle's
    op, oa = oracle.psa_build(w, chunk=1024)
    o3 = pkg.sample(torch.from_numpy(op).to(DEV), torch.from_numpy(oa.view(np.int32)).to(DEV),
                    300_001, 77, first_draw=12345)
    o4 = pkg.sample_rows(to_rows(op, oa), 300_001, 77, first_draw=12345)
    torch.cuda.synchronize()
    ref = oracle.sample(op, oa, 300_001, 77, first=12345)
    assert np.array_equal(o3.cpu().numpy().view(np.uint32), ref)
    assert np.array_equal(o4.cpu().numpy().view(np.uint32), ref)


def test_build_is_deterministic():
    n = (1 << 20) + 3
    w = inputs.lognormal(n, 2.0, 3)
    say("determinism", n)
    _, _, p1, a1 = gpu_build(w)
    _, _, p2, a2 = gpu_build(w)
    assert np.array_equal(p1, p2) and np.array_equal(a1, a2)


def test_zero_weight_items_never_drawn():
    n = 100_000
    w = inputs.uniform01(n, 2)
    w[::7] = 0.0
    say("zeros", n)
    b, st, p, a = gpu_build(w)
    r = oracle.check(w, p, a)
    assert r["zero_violations"] == 0 and r["max_rel"] <= 1e-12
    out = pkg.sample(torch.from_numpy(p).to(DEV), torch.from_numpy(a.view(np.int32)).to(DEV),
                     2_000_000, seed=1)
    drawn = out.cpu().numpy().view(np.uint32)
    assert not np.any(w[drawn] == 0.0)


@pytest.mark.parametrize("bad", ["negative", "nan", "inf", "all_zero"])
def test_invalid_weights_reported_on_device(bad):
    w = inputs.uniform01(10_000, 1)
    if bad == "negative":
        w[1234] = -1e-300
    elif bad == "nan":
        w[9999] = np.nan
    elif bad == "inf":
        w[0] = np.inf
    else:
        w[:] = 0.0
    say("invalid", bad)
    _, st, _, _ = gpu_build(w)
    assert st == pkg.ALIAS_EWEIGHTS


# --------------------------------------------------------------------------
# sampling: bit-exact with the oracle on the same table; chi-squared
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def table_2p20():
    """The oracle's table of the 2^20 uniform workload (sampled on both sides)."""
    w = inputs.make_weights("uniform_2p20")
    say("table uniform_2p20")
    p, a = oracle.psa_build(w, chunk=1024)
    return w, p, a


@pytest.mark.parametrize("count,first,table,seed", [
    (1, 0, 0, inputs.SAMPLE_SEED), (255, 0, 0, 1), (256, 3, 0, 2), (1_000_003, 0, 0, inputs.SAMPLE_SEED),
    (77_777, 2**32 - 1000, 5, 2**64 - 1), (4096 * 8 + 5, 10**9, 2**32 - 1, 0x0123456789ABCDEF)])
def test_samples_bit_exact(table_2p20, count, first, table, seed):
    w, p, a = table_2p20
    say("sample", count, first, table, seed)
    pd = torch.from_numpy(p).to(DEV)
    ad = torch.from_numpy(a.view(np.int32)).to(DEV)
    out = pkg.sample(pd, ad, count, seed, first_draw=first, table_id=table)
    torch.cuda.synchronize()
    ref = oracle.sample(p, a, count, seed, first=first, table=table)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), ref)


def test_sample_chi_squared_1e8(table_2p20):
    w, p, a = table_2p20
    say("chi2 1e8")
    pd = torch.from_numpy(p).to(DEV)
    ad = torch.from_numpy(a.view(np.int32)).to(DEV)
    counts = torch.zeros(len(w), dtype=torch.int64, device=DEV)
    per = 25_000_000
    for k in range(4):
        out = pkg.sample(pd, ad, per, inputs.SAMPLE_SEED, first_draw=k * per)
        counts += torch.bincount(out.long(), minlength=len(w))
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    assert c.sum() == 10**8
    stat, dof, pv = oracle.chi2_gof(c, 1e8 * w / w.sum())
    assert pv >= 1e-3, (stat, dof, pv)


# --------------------------------------------------------------------------
# full-size workloads, launched as the benchmark launches them
# --------------------------------------------------------------------------
def test_fullsize_powerlaw_2p27():
    cfg = inputs.WORKLOADS["powerlaw_2p27"]
    w = inputs.make_weights("powerlaw_2p27")
    say("fullsize powerlaw_2p27 build")
    b, st, p, a = gpu_build(w, cfg["chunk"])
    assert st == 0
    it = b.intermediates()
    # partition counts and split monotonicity hold at any size
    assert it["L"] + it["H"] == len(w)
    di = np.diff(it["split_i"].astype(np.int64))
    dj = np.diff(it["split_j"].astype(np.int64))
    assert np.all(di >= 0) and np.all(dj >= 0) and np.all(di + dj <= cfg["chunk"])
    say("fullsize powerlaw_2p27 oracle check")
    r = oracle.check(w, p, a)
    assert r["max_rel"] <= 1e-12 and r["zero_violations"] == 0, r
    # sampled draws across the 10^9-draw range from the oracle's table, bit-exact
    say("fullsize powerlaw_2p27 sampled draws")
    op, oa = oracle.psa_build(w, chunk=cfg["chunk"])
    rows = to_rows(op, oa)
    for first in (0, 123_456_789, 10**9 - 100_000):
        out = pkg.sample_rows(rows, 100_000, inputs.SAMPLE_SEED, first_draw=first)
        ref = oracle.sample(op, oa, 100_000, inputs.SAMPLE_SEED, first=first)
        assert np.array_equal(out.cpu().numpy().view(np.uint32), ref)


def test_fullsize_powerlaw_2p27_table_equals_oracle():
    cfg = inputs.WORKLOADS["powerlaw_2p27"]
    w = inputs.make_weights("powerlaw_2p27")
    say("fullsize powerlaw_2p27 vs oracle table")
    _, st, p, a = gpu_build(w, cfg["chunk"])
    op, oa = oracle.psa_build(w, chunk=cfg["chunk"])
    assert np.array_equal(a, oa)
    assert ulp_diff(p, op).max() <= 2


def test_fullsize_exact_integers_bitwise():
    """Exact-arithmetic weights at the full 2^27 size in the benchmark's
    launch configuration (chunk 1024, rows): every sum is exact in dd, so the
    table must equal the oracle's bit for bit, including the section splits."""
    n = 1 << 27
    say("fullsize exact 2^27")
    w = inputs.exact_integers(n, seed=2027, max_w=1 << 20, zero_frac=0.01)
    b = pkg.Builder(n, 1024, device=DEV)
    rows = b.build_rows(torch.from_numpy(w).to(DEV))
    torch.cuda.synchronize()
    assert int(b.status.item()) == 0
    pr, al = pkg.rows_split(rows)
    p = pr.cpu().numpy()
    a = al.cpu().numpy().view(np.uint32)
    op, oa, info = oracle.psa_build(w, chunk=1024, with_splits=True)
    assert np.array_equal(a, oa)
    assert np.array_equal(p, op)
    it = b.intermediates()
    assert np.array_equal(it["split_j"], info["split_j"].astype(np.uint32))
