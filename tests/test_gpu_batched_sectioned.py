"""GPU parity of batched sectioned sampling (Sec. 5 sectioned methods over a
batch of tables) through the C ABI: every table's output range equals the
CPU oracle's single-table sectioned draws with table id t, bit for bit.
Covers uneven batches with one-row, empty and draw-less tables, both table
layouts, several section sizes, thousands of tiny tables (chunks spanning
many sections), bad offsets, graph capture with the batched build, and the
full-size batched workloads on sampled tables.  The tables sampled on both
sides are built by the oracle on the CPU (uploaded for the GPU).
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


def dev_u64(a):
    return torch.from_numpy(np.asarray(a, dtype=np.uint64).view(np.int64)).to(DEV)


def oracle_tables(w, off, chunk=1024):
    """Every table of the batch built by the oracle (empty tables skipped)."""
    p = np.zeros(len(w))
    a = np.zeros(len(w), np.uint32)
    for t in range(len(off) - 1):
        s, e = int(off[t]), int(off[t + 1])
        if e > s:
            p[s:e], a[s:e] = oracle.psa_build(w[s:e], chunk=chunk)
    return p, a


def to_rows(p, a):
    r = torch.zeros((len(p), 4), dtype=torch.int32, device=DEV)
    r.view(torch.float64)[:, 0] = torch.from_numpy(p).to(DEV)
    r[:, 2] = torch.from_numpy(a.view(np.int32)).to(DEV)
    return r


def run(p, a, off, doff, seed, log2r, rows, fill=-3):
    T, total, nd = len(off) - 1, len(p), int(doff[-1])
    bs = pkg.BatchedSectionedSampler(T, total, nd, log2r, device=DEV)
    out = torch.full((max(nd, 1),), fill, dtype=torch.int32, device=DEV)[:nd]
    od, dd_ = dev_u64(off), dev_u64(doff)
    if rows:
        out, st = bs.sample_rows(to_rows(p, a), od, dd_, seed, out)
    else:
        out, st = bs.sample(torch.from_numpy(p).to(DEV), torch.from_numpy(a.view(np.int32)).to(DEV),
                            od, dd_, seed, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32), int(st.item())


def check_tables(got, p, a, off, doff, seed, log2r, tables=None):
    for t in (range(len(off) - 1) if tables is None else tables):
        s, e = int(off[t]), int(off[t + 1])
        ds, de = int(doff[t]), int(doff[t + 1])
        if de == ds:
            continue
        ref, _ = oracle.sample_sectioned(p[s:e], a[s:e], de - ds, seed, log2r, table=t)
        assert np.array_equal(got[ds:de], ref), t


@pytest.mark.parametrize("log2r", [6, 9, 13])
@pytest.mark.parametrize("rows", [False, True])
def test_batched_sectioned_bit_exact(log2r, rows):
    sizes = np.array([1, 5, 4096, 77, 30000, 64, 0, 65, 9000, 2, 20000], dtype=np.int64)
    w = inputs.batch_lognormal(sizes, seed=19, sigma=1.5)
    off = inputs.offsets_from_sizes(sizes)
    draws = inputs.apportion(500_001, sizes)
    draws[1] = 0  # a table with rows but no draws
    draws[0] = 3000  # a one-row table with many draws
    doff = inputs.offsets_from_sizes(draws)
    p, a = oracle_tables(w, off, 256)
    seed = inputs.SAMPLE_SEED + log2r
    say("batched sectioned", log2r, rows, int(doff[-1]))
    got, st = run(p, a, off, doff, seed, log2r, rows)
    assert st == 0
    check_tables(got, p, a, off, doff, seed, log2r)


def test_batched_sectioned_many_tiny_tables():
    """Thousands of tables of 1..300 rows: most output chunks span many
    sections and tables."""
    sizes = inputs.log_uniform_sizes(3000, 1, 300, seed=5)
    w = inputs.batch_lognormal(sizes, seed=6)
    off = inputs.offsets_from_sizes(sizes)
    draws = inputs.apportion(700_000, sizes)
    draws[::7] = 0
    draws[3] = 1
    doff = inputs.offsets_from_sizes(draws)
    p, a = oracle_tables(w, off, 64)
    seed = 77
    say("batched sectioned tiny", len(sizes), int(doff[-1]))
    got, st = run(p, a, off, doff, seed, 6, True)
    assert st == 0
    check_tables(got, p, a, off, doff, seed, 6)


def test_batched_sectioned_one_table_equals_single_table():
    n, count, log2r = 100_003, 1_000_001, 10
    w = inputs.power_law(n, 1.0, 4)
    p, a = oracle.psa_build(w, chunk=1024)
    off = np.array([0, n], np.uint64)
    doff = np.array([0, count], np.uint64)
    say("batched sectioned T=1")
    got, st = run(p, a, off, doff, 9, log2r, False)
    assert st == 0
    ref, _ = oracle.sample_sectioned(p, a, count, 9, log2r, table=0)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("rows", [False, True])
def test_batched_sectioned_heavy_sections(rows):
    """Sections holding far more draws than one block takes at a time (the
    shared-memory method spreads such a section over many blocks): a
    64-row table with 3 million draws, a one-row table with 400 000, counts
    on both sides of a multiple of 65536, and light tables beside them."""
    sizes = np.array([64, 1, 200, 64, 64, 5000, 64], dtype=np.int64)
    w = inputs.batch_lognormal(sizes, seed=23, sigma=2.0)
    off = inputs.offsets_from_sizes(sizes)
    draws = np.array([3_000_000, 400_000, 7, 65_536, 65_537, 131_071, 0], dtype=np.int64)
    doff = inputs.offsets_from_sizes(draws)
    p, a = oracle_tables(w, off, 64)
    seed = 4242
    say("batched sectioned heavy", rows, int(doff[-1]))
    got, st = run(p, a, off, doff, seed, 6, rows)
    assert st == 0
    check_tables(got, p, a, off, doff, seed, 6)


def test_sectioned_single_heavy_section():
    """One 64-row table (one section) with 2^22 + 3 draws through the
    single-table entry point."""
    n, count, log2r = 64, (1 << 22) + 3, 6
    w = inputs.power_law(n, 1.5, 8)
    p, a = oracle.psa_build(w, chunk=64)
    say("sectioned one heavy section", count)
    sm = pkg.SectionedSampler(n, count, log2r, device=DEV)
    counts = torch.zeros(1, dtype=torch.int64, device=DEV)
    out = sm.sample(torch.from_numpy(p).to(DEV), torch.from_numpy(a.view(np.int32)).to(DEV), 31,
                    table_id=5, counts=counts)
    torch.cuda.synchronize()
    ref, cnt = oracle.sample_sectioned(p, a, count, 31, log2r, table=5)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), ref)
    assert int(counts.item()) == count == int(np.asarray(cnt).sum())


@pytest.mark.parametrize("log2r", [14, 16])
@pytest.mark.parametrize("rows", [False, True])
def test_batched_sectioned_l2_paths(log2r, rows):
    """Sections above 2^13 rows are drawn by the L2-gathering kernel.  The
    batch makes its three chunk kinds: 2000 tiny tables with 0..2 draws
    (chunks spanning more than 256 sections), 60 mid-size tables (chunks of
    a few sections), and three tables of 2^17 + odd rows with many draws
    (chunks inside one section, starting at odd and even draw offsets)."""
    rng = np.random.default_rng(1400 + log2r)
    sizes = np.concatenate([rng.integers(1, 51, 2000), rng.integers(100, 5001, 60),
                            np.array([(1 << 17) + 3, (1 << 17) + 1001, 1 << 17])]).astype(np.int64)
    draws = np.concatenate([rng.integers(0, 3, 2000), rng.integers(100, 3001, 60),
                            np.array([300_001, 123_457, 200_000])]).astype(np.int64)
    w = inputs.batch_lognormal(sizes, seed=41, sigma=1.2)
    off = inputs.offsets_from_sizes(sizes)
    doff = inputs.offsets_from_sizes(draws)
    p, a = oracle_tables(w, off, 512)
    seed = 5151 + log2r
    say("batched sectioned L2 paths", log2r, rows, int(doff[-1]))
    got, st = run(p, a, off, doff, seed, log2r, rows)
    assert st == 0
    check_tables(got, p, a, off, doff, seed, log2r)


def test_batched_sectioned_bad_tables():
    sizes = [10, 0, 20]
    w = inputs.uniform01(30, 2)
    off = inputs.offsets_from_sizes(sizes)
    p, a = oracle_tables(w, off, 64)
    # table 1 is empty but gets draws: EINVAL, its draws 0xFFFFFFFF, the others exact
    doff = inputs.offsets_from_sizes([5, 3, 4])
    say("batched sectioned bad table")
    got, st = run(p, a, off, doff, 1, 6, True)
    assert st == pkg.ALIAS_EINVAL
    assert (got[5:8] == 0xFFFFFFFF).all()
    check_tables(got, p, a, off, doff, 1, 6, tables=[0, 2])
    # an empty table without draws is fine
    doff = inputs.offsets_from_sizes([5, 0, 4])
    got, st = run(p, a, off, doff, 1, 6, False)
    assert st == 0
    check_tables(got, p, a, off, doff, 1, 6)


@pytest.mark.parametrize("case", ["draw_end", "item_end", "decreasing", "draw_start"])
def test_batched_sectioned_inconsistent_offsets(case):
    sizes = [10, 7, 20]
    w = inputs.uniform01(37, 3)
    off = inputs.offsets_from_sizes(sizes).astype(np.uint64)
    p, a = oracle_tables(w, off, 64)
    doff = inputs.offsets_from_sizes([5, 3, 4]).astype(np.uint64)
    nd = 12
    if case == "draw_end":
        doff[-1] = 11
    elif case == "item_end":
        off[-1] = 36
    elif case == "decreasing":
        doff[1], doff[2] = 9, 6
    else:
        doff[0] = 1
    T = 3
    say("batched sectioned inconsistent", case)
    bs = pkg.BatchedSectionedSampler(T, 37, nd, 6, device=DEV)
    out = torch.zeros(nd, dtype=torch.int32, device=DEV)
    rows, od, dd_ = to_rows(p, a), dev_u64(off), dev_u64(doff)  # alive until synchronised
    st = pkg.lib().alias_sample_batched_sectioned_rows(
        rows.data_ptr(), od.data_ptr(), T, 37, dd_.data_ptr(), nd, 5, 6, out.data_ptr(),
        bs.ws.data_ptr(), bs.ws_bytes, bs.status.data_ptr(), None)
    torch.cuda.synchronize()
    assert st == 0
    assert int(bs.status.item()) == pkg.ALIAS_EINVAL
    assert (out.cpu().numpy().view(np.uint32) == 0xFFFFFFFF).all()


def test_batched_sectioned_zero_draws_and_bad_arguments():
    L = pkg.lib()
    assert L.alias_sample_batched_sectioned_workspace_bytes(0, 10, 10, 8) == 0
    assert L.alias_sample_batched_sectioned_workspace_bytes(3, 0, 10, 8) == 0
    assert L.alias_sample_batched_sectioned_workspace_bytes(3, 10, 10, 5) == 0
    assert L.alias_sample_batched_sectioned_workspace_bytes(3, 10, 10, 32) == 0
    assert L.alias_sample_batched_sectioned_workspace_bytes(3, 10, (1 << 40) + 1, 8) == 0
    sizes = [3, 4]
    w = inputs.uniform01(7, 4)
    off = inputs.offsets_from_sizes(sizes)
    p, a = oracle_tables(w, off, 64)
    say("batched sectioned zero draws")
    got, st = run(p, a, off, np.zeros(3, np.uint64), 1, 6, True)
    assert st == 0 and got.size == 0


def test_batched_sectioned_graph_capture():
    """Batched build and batched sectioned sampling captured in one graph:
    every replay equals the eager result; the eager draws equal the oracle's
    on the eager tables' oracle twins where those tables are bit-exact."""
    sizes = inputs.log_uniform_sizes(400, 16, 30000, seed=24)
    w1 = inputs.batch_lognormal(sizes, seed=25)
    w2, _ = inputs.batch_zipf(sizes, seed=26)
    off = inputs.offsets_from_sizes(sizes)
    doff = inputs.offsets_from_sizes(inputs.apportion(1 << 21, sizes))
    T, total, nd = len(sizes), len(w1), int(doff[-1])
    say("batched sectioned graph", T, total, nd)
    bb = pkg.BatchBuilder(T, total, 1024, device=DEV)
    bs = pkg.BatchedSectionedSampler(T, total, nd, 10, device=DEV)
    wd = torch.from_numpy(w1).to(DEV)
    od, dd_ = dev_u64(off), dev_u64(doff)
    rows = torch.empty((total, 4), dtype=torch.int32, device=DEV)
    out = torch.empty(nd, dtype=torch.int32, device=DEV)
    seed = 4242

    def step():
        bb.build_rows(wd, od, rows=rows)
        bs.sample_rows(rows, od, dd_, seed, out)

    refs = []
    for w in (w1, w2):
        wd.copy_(torch.from_numpy(w))
        step()
        torch.cuda.synchronize()
        refs.append((rows.clone(), out.clone()))
    wd.copy_(torch.from_numpy(w1))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for k, which in enumerate((0, 1, 1, 0)):
        rows.fill_(-1)
        out.fill_(-1)
        bs.status.fill_(99)
        wd.copy_(torch.from_numpy((w1, w2)[which]))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert (bb.status == 0).all(), k
        assert int(bs.status.item()) == 0, k
        assert torch.equal(rows, refs[which][0]), k
        assert torch.equal(out, refs[which][1]), k
        _ = (out.float().sum() + 1).item()  # eager work between replays
    # the eager draws of sampled tables against the oracle on the same tables
    pr, al = pkg.rows_split(refs[0][0])
    p = pr.cpu().numpy()
    a = al.cpu().numpy().view(np.uint32)
    for t in (0, 17, T - 1):
        s_, e = int(off[t]), int(off[t + 1])
        op, oa = oracle.psa_build(w1[s_:e], chunk=1024)
        if np.array_equal(op, p[s_:e]) and np.array_equal(oa, a[s_:e]):
            check_tables(refs[0][1].cpu().numpy().view(np.uint32), p, a, off, doff, seed, 10,
                         tables=[t])


@pytest.mark.parametrize("name,log2r", [("batch_100k_16_65536", 13), ("batch_1024_2p14_2p22", 13)])
def test_batched_sectioned_full_size(name, log2r):
    """The batched workloads at full size, sampled in the benchmark's
    configuration; sampled tables hold oracle-built rows and their whole
    output ranges are bit-exact with the oracle."""
    say("full batched sectioned", name, "generating")
    w, off, doff = inputs.make_batch(name)
    T, total, nd = len(off) - 1, len(w), int(doff[-1])
    say("full batched sectioned", name, T, total, nd)
    bb = pkg.BatchBuilder(T, total, 1024, device=DEV)
    od, dd_ = dev_u64(off), dev_u64(doff)
    wd = torch.from_numpy(w).to(DEV)
    rows = bb.build_rows(wd, od)
    del wd
    torch.cuda.synchronize()
    assert (bb.status == 0).all()
    sizes = np.diff(off.astype(np.int64))
    rng = np.random.default_rng(2)
    picks = sorted(set(rng.integers(0, T, size=5).tolist()) | {0, T - 1, int(np.argmax(sizes))})
    tabs = {}
    for t in picks:
        s, e = int(off[t]), int(off[t + 1])
        op, oa = oracle.psa_build(w[s:e], chunk=1024)
        tabs[t] = (op, oa)
        rows[s:e] = to_rows(op, oa)
    del w
    bs = pkg.BatchedSectionedSampler(T, total, nd, log2r, device=DEV)
    out = torch.empty(nd, dtype=torch.int32, device=DEV)
    seed = inputs.SAMPLE_SEED
    out, st = bs.sample_rows(rows, od, dd_, seed, out)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    for t in picks:
        ds, de = int(doff[t]), int(doff[t + 1])
        op, oa = tabs[t]
        ref, _ = oracle.sample_sectioned(op, oa, de - ds, seed, log2r, table=t)
        assert np.array_equal(out[ds:de].cpu().numpy().view(np.uint32), ref), t


def test_batched_sectioned_chi_squared():
    """Batched sectioned draws of a few tables (4e7 draws in all, sections of
    2^8 rows) fit each table's w / W (grouped chi-squared per table)."""
    sizes = np.array([300, 70_000, 5000, 1], dtype=np.int64)
    w = inputs.batch_lognormal(sizes, seed=61, sigma=1.0)
    off = inputs.offsets_from_sizes(sizes)
    draws = np.array([3_000_000, 30_000_000, 6_999_999, 1], dtype=np.int64)
    doff = inputs.offsets_from_sizes(draws)
    p, a = oracle_tables(w, off, 256)
    say("batched sectioned chi2")
    got, st = run(p, a, off, doff, 4321, 8, True)
    assert st == 0
    for t in range(len(sizes)):
        s, e = int(off[t]), int(off[t + 1])
        ds, de = int(doff[t]), int(doff[t + 1])
        c = np.bincount(got[ds:de].astype(np.int64), minlength=e - s)
        assert c.size == e - s and c.sum() == de - ds
        if e - s > 1:
            stat, dof, pv = oracle.chi2_gof(c, (de - ds) * w[s:e] / w[s:e].sum())
            assert pv >= 1e-3, (t, stat, dof, pv)


def test_max_tables_build_and_sample():
    """The largest batch the ABI takes: 2^20 tables of 1..3 items, built in
    one batch and sampled plain and sectioned; sampled tables against the
    oracle (tables bit for bit on exact inputs, draws bit for bit)."""
    T = 1 << 20
    rng = np.random.default_rng(77)
    sizes = rng.integers(1, 4, T).astype(np.int64)
    w = rng.integers(1, 1 << 20, int(sizes.sum())).astype(np.float64)
    off = inputs.offsets_from_sizes(sizes)
    # make every table's total a multiple of its size: W/n is then an integer
    # and every sum of the build is exact, so tables compare bit for bit
    last = off[1:].astype(np.int64) - 1
    tot = np.add.reduceat(w, off[:-1].astype(np.int64))
    w[last] += (-tot) % sizes
    draws = rng.integers(0, 4, T).astype(np.int64)
    doff = inputs.offsets_from_sizes(draws)
    total, nd = len(w), int(doff[-1])
    say("max tables", T, total, nd)
    od, dd_ = dev_u64(off), dev_u64(doff)
    bb = pkg.BatchBuilder(T, total, 64, device=DEV)
    rows = bb.build_rows(torch.from_numpy(w).to(DEV), od)
    out_p = torch.empty(nd, dtype=torch.int32, device=DEV)
    out_p, sst = pkg.sample_batched_rows(rows, od, dd_, 5, out_p)
    bs = pkg.BatchedSectionedSampler(T, total, nd, 6, device=DEV)
    out_s = torch.empty(nd, dtype=torch.int32, device=DEV)
    out_s, sst2 = bs.sample_rows(rows, od, dd_, 5, out_s)
    torch.cuda.synchronize()
    assert (bb.status == 0).all() and int(sst.item()) == 0 and int(sst2.item()) == 0
    pr, al = pkg.rows_split(rows)
    p = pr.cpu().numpy()
    a = al.cpu().numpy().view(np.uint32)
    gp, gs = out_p.cpu().numpy().view(np.uint32), out_s.cpu().numpy().view(np.uint32)
    for t in sorted(set(rng.integers(0, T, 300).tolist()) | {0, T - 1}):
        s, e = int(off[t]), int(off[t + 1])
        op, oa = oracle.psa_build(w[s:e], chunk=64)
        assert np.array_equal(p[s:e], op) and np.array_equal(a[s:e], oa), t
        ds, de = int(doff[t]), int(doff[t + 1])
        if de > ds:
            assert np.array_equal(gp[ds:de], oracle.sample(op, oa, de - ds, 5, first=0, table=t)), t
            ref, _ = oracle.sample_sectioned(op, oa, de - ds, 5, 6, table=t)
            assert np.array_equal(gs[ds:de], ref), t


@pytest.mark.parametrize("case", range(40))
def test_random_small_batches(case):
    """Random small batches (empty tables, one-row tables, ragged sizes,
    tables without draws, every section size and chunk): exact-arithmetic
    weights, so each table equals the oracle's bit for bit; plain and
    sectioned batched draws equal the oracle's per table."""
    rng = np.random.default_rng(1000 + case)
    T = int(rng.integers(1, 60))
    sizes = rng.integers(0, 3000, T).astype(np.int64)
    sizes[rng.random(T) < 0.15] = 0
    sizes[rng.random(T) < 0.15] = 1
    if sizes.sum() == 0:
        sizes[0] = 5
    off = inputs.offsets_from_sizes(sizes)
    w = rng.integers(0, 1 << 16, int(sizes.sum())).astype(np.float64)
    for t in range(T):  # positive totals divisible by the table size: exact W/n
        s, e = int(off[t]), int(off[t + 1])
        if e > s:
            w[e - 1] += 1 + (-(w[s:e].sum() + 1)) % (e - s)
    draws = np.where(sizes > 0, rng.integers(0, 20_000, T), 0).astype(np.int64)
    draws[rng.random(T) < 0.2] = 0
    doff = inputs.offsets_from_sizes(draws)
    chunk = int(2 ** rng.integers(6, 12))
    log2r = int(rng.integers(6, 14))
    seed = int(rng.integers(0, 2**63))
    total, nd = len(w), int(doff[-1])
    say("random batch", case, T, total, nd, chunk, log2r)
    od, dd_ = dev_u64(off), dev_u64(doff)
    bb = pkg.BatchBuilder(T, total, chunk, device=DEV)
    rows = bb.build_rows(torch.from_numpy(w).to(DEV), od)
    outp = torch.full((max(nd, 1),), -5, dtype=torch.int32, device=DEV)[:nd]
    bs = pkg.BatchedSectionedSampler(T, total, nd, log2r, device=DEV)
    outs = torch.full((max(nd, 1),), -5, dtype=torch.int32, device=DEV)[:nd]
    if nd:
        outp, sp = pkg.sample_batched_rows(rows, od, dd_, seed, outp)
    outs, ss = bs.sample_rows(rows, od, dd_, seed, outs)
    torch.cuda.synchronize()
    st = bb.status.cpu().numpy()
    pr, al = pkg.rows_split(rows)
    p = pr.cpu().numpy()
    a = al.cpu().numpy().view(np.uint32)
    gp, gs = outp.cpu().numpy().view(np.uint32), outs.cpu().numpy().view(np.uint32)
    assert int(ss.item()) == 0
    if nd:
        assert int(sp.item()) == 0
    for t in range(T):
        s, e = int(off[t]), int(off[t + 1])
        ds, de = int(doff[t]), int(doff[t + 1])
        if e == s:
            assert st[t] == pkg.ALIAS_EINVAL  # an empty table is reported, not built
            continue
        assert st[t] == 0, t
        op, oa = oracle.psa_build(w[s:e], chunk=chunk)
        assert np.array_equal(p[s:e], op) and np.array_equal(a[s:e], oa), t
        if de > ds:
            assert np.array_equal(gp[ds:de], oracle.sample(op, oa, de - ds, seed, first=0, table=t)), t
            ref, _ = oracle.sample_sectioned(op, oa, de - ds, seed, log2r, table=t)
            assert np.array_equal(gs[ds:de], ref), t
