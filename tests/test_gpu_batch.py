"""The batched form: uneven boxes stepped in one captured HIP graph give exactly the results of
stepping each box alone, and those match the oracle."""
import numpy as np
import pytest
import torch

import paper_1601_00035_amd as nslgf
import workloads
from oracle import ifherk

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _problem(n, seed, dtype):
    n, dx, ring, re, cfl = workloads.small_ring_case(n, seed)
    w = workloads.ring_edge_vorticity(n, dx, ring, quad=2)
    u0 = nslgf.vor2vel(torch.from_numpy(w).to(DEV), dx)
    dt = cfl * dx / nslgf.max_cell_speed(u0)
    return u0.to(dtype), dx, dt, re


@pytest.mark.parametrize("mode", [nslgf.BATCH_PASSES, nslgf.BATCH_PER_PROBLEM])
def test_batched_equals_unbatched_bitwise(mode):
    """Both forms of the batch graph (batched passes over groups of like problems, or one branch per
    problem) give the one-by-one results bit for bit over three replays.  The specs hold groups of equal
    boxes (two 24^3 FP64 problems with the same step parameters share every launch) and singletons; 128^3
    in FP32 and FP64 pads to 256, where the column passes use the wide and the narrow plan."""
    specs = [(24, 1, torch.float64), (32, 2, torch.float64), (20, 3, torch.float32), (28, 4, torch.float64),
             (24, 5, torch.float32), (128, 6, torch.float32), (128, 7, torch.float64), (24, 1, torch.float64),
             (32, 2, torch.float64)]
    probs = [_problem(*s) for s in specs]
    solo = [nslgf.HerkState(u.clone(), dx, dt, re, "A", n_buf=2) for (u, dx, dt, re) in probs]
    batch = [nslgf.HerkState(u.clone(), dx, dt, re, "A", n_buf=2) for (u, dx, dt, re) in probs]
    nslgf.set_batch_mode(mode)
    try:
        for step in range(3):  # the first call captures, the next ones replay the graph
            for st in solo:
                st.step()
            nslgf.herk_step_batched(batch)
            torch.cuda.synchronize()
            for a, b in zip(solo, batch):
                assert torch.equal(a.u, b.u), step
                assert torch.equal(a.d, b.d), step
                assert a.t == b.t
        groups, launches = nslgf.batch_info()
        if mode == nslgf.BATCH_PASSES:
            # the repeated specs share their group: 9 problems in 7 groups, and fewer launches than the
            # per-problem form's 9 x (launches of one step)
            assert groups == 7, groups
        else:
            assert groups == 0
    finally:
        nslgf.set_batch_mode(nslgf.BATCH_PASSES)


def test_batched_passes_fall_back_for_the_guard():
    """A guarded step has a kernel without a batched form: the batch is captured per problem and still
    equals one-by-one steps."""
    u, dx, dt, re = _problem(24, 11, torch.float64)
    a = nslgf.HerkState(u.clone(), dx, dt, re, "A", n_buf=2, guard=True)
    b = nslgf.HerkState(u.clone(), dx, dt, re, "A", n_buf=2, guard=True)
    a.step()
    nslgf.herk_step_batched([b])
    assert torch.equal(a.u, b.u) and nslgf.batch_info()[0] == 0


def test_batched_matches_oracle_and_recaptures():
    u, dx, dt, re = _problem(24, 7, torch.float64)
    u2, dx2, dt2, re2 = _problem(16 + 8, 8, torch.float64)
    u0 = u.cpu().numpy()
    ref, dref = ifherk.step(u0, dt, dx, re, "A", n_buf=2)
    states = [nslgf.HerkState(u.clone(), dx, dt, re, "A", n_buf=2), nslgf.HerkState(u2.clone(), dx2, dt2, re2, "B")]
    nslgf.herk_step_batched(states)
    got = states[0].u.cpu().numpy()
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-12
    assert np.abs(states[0].d.cpu().numpy() - dref).max() / np.abs(dref).max() < 1e-12
    # a new dt changes the captured coefficients: the batch is captured again
    states[0].set_dt(dt / 2)
    solo = nslgf.HerkState(states[0].u.clone(), dx, dt / 2, re, "A", n_buf=2)
    solo.step()
    nslgf.herk_step_batched(states)
    assert torch.equal(solo.u, states[0].u)


def test_batched_rejects_shared_buffers():
    u, dx, dt, re = _problem(16 + 4, 9, torch.float64)
    st = nslgf.HerkState(u, dx, dt, re)
    with pytest.raises(nslgf.NslgfError):
        nslgf.herk_step_batched([st, st])


def test_table_rebuild_recaptures_the_batch_graph():
    """lgf_table rebuilds a box's plan (a new spectrum buffer); a batch captured before must not replay
    with the freed spectrum: the next batched step is captured again and equals a plain step."""
    u, dx, dt, re = _problem(24, 10, torch.float64)
    st = nslgf.HerkState(u.clone(), dx, dt, re, "A", n_buf=2)
    nslgf.herk_step_batched([st])
    nslgf.lgf_table(24, 24, 24, torch.float64)
    # allocations after the rebuild may land on the freed spectrum's memory; write over them
    junk = [torch.full((24 ** 3 * 8,), float("nan"), dtype=torch.float64, device=DEV) for _ in range(4)]
    solo = nslgf.HerkState(st.u.clone(), dx, dt, re, "A", n_buf=2)
    solo.step()
    nslgf.herk_step_batched([st])
    torch.cuda.synchronize()
    assert torch.equal(solo.u, st.u) and torch.equal(solo.d, st.d)
    del junk
