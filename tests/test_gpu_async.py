"""Asynchronous slots: every slot runs whole passes back to back inside one launch and takes new
instances from the device queue as its own finish (iteration-level batching, Sec. V, without a
grid-wide step between passes).  An instance's arithmetic does not depend on the slot or the
pass that runs it, so the results must equal those of the per-pass kernels bit for bit, also
when instances outnumber slots, with the FP32 factor, and across restoration phases."""
import numpy as np
import pytest

from paper_2606_26341_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _solve(torch, w, TH, slots, **opts):
    from paper_2606_26341_amd import hipipm
    s = hipipm.Solver(w, slots, hipipm.default_options(**opts))
    out = {k: v.cpu().numpy() for k, v in s.solve(TH).items()}
    return out, s.stats()


@pytest.mark.parametrize("name,n_inst,slots,prec", [
    ("C1", 512, 512, 0),     # one instance per slot
    ("C1", 700, 96, 0),      # refills from the queue, ragged last wave
    ("C2", 384, 128, 0),     # restoration phases and second-order corrections
    ("C2", 256, 64, 1),      # FP32 factor with FP64 refinement
])
@pytest.mark.parametrize("passes", [1, 7])
def test_async_slots_match_pass_kernels(torch_cuda, name, n_inst, slots, prec, passes):
    torch = torch_cuda
    w = W.get(name)
    TH = torch.tensor(w.thetas(0, n_inst), dtype=torch.float64, device="cuda")
    say(name, n_inst, "instances", slots, "slots, precision", prec, "async passes", passes)
    ref, st_ref = _solve(torch, w, TH, slots, precision=prec)
    got, st = _solve(torch, w, TH, slots, precision=prec, async_passes=passes)
    for k in ref:
        assert np.array_equal(ref[k], got[k], equal_nan=True), k
    for k in ("iterations", "resto_iterations", "resto_entries", "soc_tried", "soc_accepted",
              "factorizations"):
        assert st[k] == st_ref[k], k
    say("statuses", np.bincount(got["status"], minlength=6), "iterations", st["iterations"])


@pytest.mark.parametrize("prec", [0, 1])
def test_resident_slots_single_launch_matches_pass_kernels(torch_cuda, prec):
    """hipipm_resident_slots: a whole number of workgroups per compute unit (at least one); a
    solve through exactly that many slots with an unbounded pass count (one launch, every slot
    resident, instances outnumbering the slots) equals the per-pass kernels bit for bit."""
    torch = torch_cuda
    from paper_2606_26341_amd import hipipm
    w = W.get("C2")
    n = hipipm.resident_slots(w, hipipm.default_options(precision=prec))
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    say("resident slots", n, "compute units", cus, "precision", prec)
    assert n >= cus and n % cus == 0
    TH = torch.tensor(w.thetas(0, n + n // 2 + 7), dtype=torch.float64, device="cuda")
    ref, st_ref = _solve(torch, w, TH, n, precision=prec)
    got, st = _solve(torch, w, TH, n, precision=prec, async_passes=1 << 20)
    for k in ref:
        assert np.array_equal(ref[k], got[k], equal_nan=True), k
    assert st["iterations"] == st_ref["iterations"]
