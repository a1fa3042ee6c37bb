"""The allocation-free time-step query (mhd_dt_noalloc) against the context
entry point mhd_dt on the same states, through the C ABI: two calls in a row
on one GPU, the second with a smaller box (the shared scratch array still
holds the first call's partials), plus a 2D box and a box with outflow walls.
Both compute the same per-cell rates and take an exact maximum, so the steps
must be equal bit for bit."""
import numpy as np
import pytest

from paper_2606_12753_amd import mhd
from paper_2606_12753_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mhd.load()


def _dt_ref(spec, st):
    with mhd.Sim([spec]) as sim:
        sim.set_state(0, st.cons, st.bface, 0.0)
        return sim.dt(0)[0]


def test_dt_noalloc_equals_dt_on_consecutive_calls():
    import torch
    cases = [W.blast_3d(n=64), W.random_smooth(n=(20, 16, 12), seed=92, bc=(0, 1, 0)),
             W.orszag_tang_2d(n=40), W.random_smooth(n=(9, 7, 5), seed=93, bc=(1, 1, 1))]
    out = torch.full((len(cases),), -1.0, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    for k, wl in enumerate(cases):
        spec, st = wl.boxes[0], wl.states[0]
        ref = _dt_ref(spec, st)
        dc = [torch.from_numpy(a).cuda() for a in st.cons]
        db = [torch.from_numpy(a).cuda() for a in st.bface]
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            mhd.dt_noalloc(spec, dc, db, out[k:k + 1], stream=stream)
        stream.synchronize()
        got = float(out[k].item())
        print(f"[no-alloc dt] {wl.name} {tuple(spec.n)}: {got!r} vs mhd_dt {ref!r}", flush=True)
        assert got == ref, (wl.name, got, ref)
    # the same large box again after the small ones: same value
    spec, st = cases[0].boxes[0], cases[0].states[0]
    dc = [torch.from_numpy(a).cuda() for a in st.cons]
    db = [torch.from_numpy(a).cuda() for a in st.bface]
    again = torch.empty(1, dtype=torch.float64, device="cuda")
    mhd.dt_noalloc(spec, dc, db, again)
    torch.cuda.synchronize()
    assert float(again.item()) == float(out[0].item())


def test_dt_noalloc_nonphysical_cell_gives_zero():
    import torch
    wl = W.random_smooth(n=(12, 10, 8), seed=94)
    spec, st = wl.boxes[0], wl.states[0]
    cons = [torch.from_numpy(a.copy()).cuda() for a in st.cons]
    cons[0][2, 3, 4] = -1.0
    db = [torch.from_numpy(a).cuda() for a in st.bface]
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    mhd.dt_noalloc(spec, cons, db, out)
    torch.cuda.synchronize()
    assert float(out.item()) == 0.0
