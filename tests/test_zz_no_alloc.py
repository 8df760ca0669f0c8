"""The allocation-free entry point of fast entry selection: pa_select_entries_noalloc,
called through the C-ABI, gives the same entries and distances as pa_select_entries on
two calls in a row (the second smaller, over what the first left in the static scratch),
matches the oracle to the usual bar, allocates no device memory, and refuses more queries
than its static scratch holds."""

import numpy as np
import pytest

import oracle
import paper_2503_21206_amd as pa
from tests.gpu_checks import _t, say
from tests.parity import TIE, DistTally
from tests.workload import build_tiny, device_tables, oracle_entries

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pa.device_init(0)
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def tiny():
    return build_tiny(device="cpu")


def _oracle_check(ids, d, oi, od, margin):
    tally = DistTally()
    bad = 0
    for i in range(ids.shape[0]):
        if not (ids[i] == oi[i]).all():
            assert margin[i] <= TIE, (i, ids[i], oi[i], margin[i])
            bad += 1
            continue
        tally.check(d[i], od[i], i)
    tally.done()
    assert bad <= max(1, ids.shape[0] // 1000)


def test_noalloc_entry_selection_matches_the_allocating_call(dev, tiny):
    EV, EVn, EVid = device_tables(tiny)
    EVd, EVnd, EVidd = _t(EV, dev), _t(EVn, dev), _t(EVid, dev)
    E = 8
    _, _, cl_all, _ = oracle_entries(tiny, E)
    for m, lo in ((1000, 0), (137, 500)):  # the second call is smaller and starts elsewhere
        say(f"select_entries_noalloc: {m} queries (rows {lo}..{lo + m - 1}) against select_entries and the oracle")
        Qr = tiny["Qr32"][lo:lo + m]
        Qd = _t(Qr, dev)
        cld = _t(cl_all[lo:lo + m].astype(np.int32), dev)
        ids = torch.full((m, E), -7, dtype=torch.int32, device=dev)
        dist = torch.full((m, E), -7.0, dtype=torch.float32, device=dev)
        pa.select_entries_noalloc(Qd, cld, EVd, EVnd, EVidd, ids, dist, E)
        ref_ids, ref_d = pa.select_entries(Qd, cld, EVd, EVnd, EVidd, E)
        torch.cuda.synchronize()
        a_i, a_d = ids.cpu().numpy(), dist.cpu().numpy()
        b_i, b_d = ref_ids.cpu().numpy(), ref_d.cpu().numpy()
        assert (a_i == b_i).all() and (a_d.view(np.uint32) == b_d.view(np.uint32)).all()
        oi, od, _, margin = oracle.select_entries(Qr, tiny["cent32"].astype(np.float64), tiny["buckets"],
                                                  tiny["P32"], tiny["pivots"], E)
        _oracle_check(a_i, a_d, oi, od, margin)


def test_noalloc_entry_selection_allocates_nothing_and_bounds_its_input(dev, tiny):
    EV, EVn, EVid = device_tables(tiny)
    EVd, EVnd, EVidd = _t(EV, dev), _t(EVn, dev), _t(EVid, dev)
    E, m = 8, 512
    _, _, cl, _ = oracle_entries(tiny, E, tiny["Qr32"][:m])
    Qd, cld = _t(tiny["Qr32"][:m], dev), _t(cl.astype(np.int32), dev)
    ids = torch.empty((m, E), dtype=torch.int32, device=dev)
    dist = torch.empty((m, E), dtype=torch.float32, device=dev)
    pa.select_entries_noalloc(Qd, cld, EVd, EVnd, EVidd, ids, dist, E)  # kernels loaded
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info(dev)
    for _ in range(3):
        pa.select_entries_noalloc(Qd, cld, EVd, EVnd, EVidd, ids, dist, E)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info(dev)
    say(f"device memory free before / after three calls: {free0} / {free1}")
    assert free1 == free0
    say("more queries than the static scratch holds: refused before any launch")
    big = 262_145
    Qb = torch.zeros((big, tiny["spec"].d_r), dtype=torch.float32, device=dev)
    clb = torch.zeros((big,), dtype=torch.int32, device=dev)
    ib = torch.empty((big, E), dtype=torch.int32, device=dev)
    db = torch.empty((big, E), dtype=torch.float32, device=dev)
    with pytest.raises(pa.PilotannError) as e:
        pa.select_entries_noalloc(Qb, clb, EVd, EVnd, EVidd, ib, db, E)
    assert e.value.status == -1 and "262144" in str(e.value)
