"""bst_execute_static (the entry point for callers that cannot allocate):
through the C ABI it gives bst_execute's result bit for bit, on two calls in
a row with the second operator smaller than the first, and the oracle's
result within the form's tolerance; a plan whose workspace exceeds the
static array is refused before anything is enqueued."""
import numpy as np
import pytest

from tests.gpu_common import DEV, check, dev, heff_operands, host, require_gpu, torch
from oracle import oracle as orc
from paper_2401_01921_amd import bst, workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_execute_static_matches_execute(prec):
    for chi, qmax in ((512, 8), (256, 6)):   # the second call's operator is smaller
        specs, O = heff_operands(2, chi=chi, qmax=qmax)
        T = {n: bst.Tensor(*s) for n, s in specs.items()}
        plan = bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], prec)
        assert plan.workspace_bytes <= bst.STATIC_WORKSPACE_BYTES
        ins = [dev(O[n].data) for n in ("L", "W1", "W2", "R", "psi")]
        want = torch.full((O["psi"].numel,), np.nan, dtype=torch.float64, device=DEV)
        ws = bst.workspace(plan.workspace_bytes)
        ws.fill_(255)
        plan.execute(ins, [want], ws)
        got = torch.full((O["psi"].numel,), np.nan, dtype=torch.float64, device=DEV)
        print("static execute", prec, chi, plan.workspace_bytes, flush=True)
        plan.execute_static(ins, [got])
        torch.cuda.synchronize()
        assert np.array_equal(host(got), host(want)), (prec, chi)
        ref = orc.heff_apply(O["L"], O["W1"], O["W2"], O["R"], O["psi"]).data
        check(host(got), ref, prec, f"static execute chi {chi}")


def test_execute_static_refuses_large_plans():
    v = wl.gaussian_sector_dims(4096, 20)
    T = {k: bst.Tensor(*s) for k, s in wl.heff_specs("1", v, v).items()}
    plan = bst.heff_plan(T["L"], T["W1"], T["W2"], T["R"], T["psi"], "fp64")
    assert plan.workspace_bytes > bst.STATIC_WORKSPACE_BYTES
    ins = [torch.empty(n, dtype=torch.float64, device=DEV) for n in plan.in_numel]
    out = torch.empty(plan.out_numel[0], dtype=torch.float64, device=DEV)
    with pytest.raises(bst.BstError) as err:
        plan.execute_static(ins, [out])
    assert err.value.status == "E_INVALID" and "static" in str(err.value)
