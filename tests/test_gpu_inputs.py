"""GPU checks of input handling through the C-ABI: the opt-in device check of neutrality and
finiteness (PSWFE_CHECK_INPUT; the k = 0 mode is dropped, Sec. 3.1.2), the NaN that a non-finite
position carries into the outputs without it, and refusal of the check under graph capture."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pw = pytest.importorskip("paper_2602_16591_amd")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def tdev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev())


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_check_passes_neutral_finite_input_and_changes_nothing(prec):
    dt = torch.float32 if prec == "fp32" else torch.float64
    x, q, L = W.uniform_pm1(2000, seed=61)
    c = pw.choose_params(1e-6, L, m=32)
    plan = pw.Plan(c, prec, n_max=len(q))
    X, Q = tdev(x, dt), tdev(q, dt)
    p0, F0, E0 = plan.compute(X, Q)
    p1, F1, E1 = plan.compute(X, Q, check=True)
    tol = 1e-5 if prec == "fp32" else 1e-12
    assert float((p1 - p0).abs().max()) <= tol * float(p0.abs().max())
    assert float((F1 - F0).abs().max()) <= tol * float(F0.abs().max())
    assert abs(float(E1[0]) - float(E0[0])) <= tol * abs(float(E0[0]))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_check_reports_a_net_charge_and_leaves_outputs(prec):
    dt = torch.float32 if prec == "fp32" else torch.float64
    x, q, L = W.uniform_pm1(1000, seed=62)
    q = q.copy()
    q[0] += 0.01            # net charge 0.01 against sum |q| = 1000: 1e-5 > 1e-6
    c = pw.choose_params(1e-6, L, m=24)
    plan = pw.Plan(c, prec, n_max=len(q))
    phi = torch.full((len(q),), 7.0, dtype=dt, device=dev())
    with pytest.raises(pw.PswfeError) as e:
        plan.compute(tdev(x, dt), tdev(q, dt), phi=phi, check=True)
    assert e.value.status == pw.E_NONNEUTRAL
    assert bool((phi == 7.0).all())
    # without the check the call runs (the uniform background is implied)
    out, _, _ = plan.compute(tdev(x, dt), tdev(q, dt))
    assert bool(torch.isfinite(out).all())


@pytest.mark.parametrize("what", ["nan_position", "inf_position", "inf_charge", "nan_charge"])
def test_check_reports_non_finite_input(what):
    x, q, L = W.uniform_pm1(500, seed=63)
    x, q = x.copy(), q.copy()
    if what == "nan_position":
        x[11, 2] = np.nan
    elif what == "inf_position":
        x[12, 0] = -np.inf
    elif what == "inf_charge":
        q[13] = np.inf
    else:
        q[14] = np.nan
    c = pw.choose_params(1e-6, L, m=20)
    plan = pw.Plan(c, "fp64", n_max=len(q))
    with pytest.raises(pw.PswfeError) as e:
        plan.compute(tdev(x, torch.float64), tdev(q, torch.float64), check=True)
    assert e.value.status == pw.E_NONFINITE
    # unchecked: NaN everywhere rather than a silent, finite, wrong answer
    phi, F, E = plan.compute(tdev(x, torch.float64), tdev(q, torch.float64))
    assert bool(torch.isnan(phi).all()) and bool(torch.isnan(F).all()) and bool(torch.isnan(E).all())


def test_check_per_system_of_a_batch():
    systems = [W.uniform_pm1(300, seed=64), W.uniform_pm1(500, seed=65, L=1.3)]
    params = [pw.choose_params(1e-6, L, m=20) for _, _, L in systems]
    plan = pw.BatchPlan(params, [len(q) for _, q, _ in systems], "fp32")
    x = np.concatenate([s[0] for s in systems])
    q = np.concatenate([s[1] for s in systems])
    X, Q = tdev(x, torch.float32), tdev(q, torch.float32)
    plan.compute(X, Q, check=True)                 # both neutral
    q2 = q.copy()
    q2[300] += 2.0                                 # second system: net charge +2
    with pytest.raises(pw.PswfeError) as e:
        plan.compute(X, tdev(q2, torch.float32), check=True)
    assert e.value.status == pw.E_NONNEUTRAL
    # a pair of opposite net charges in two systems is still caught per system
    q3 = q.copy()
    q3[0] += 0.5
    q3[300] -= 0.5
    with pytest.raises(pw.PswfeError) as e:
        plan.compute(X, tdev(q3, torch.float32), check=True)
    assert e.value.status == pw.E_NONNEUTRAL


def test_check_is_refused_under_graph_capture():
    """The check reads its result back on the host, which a captured stream cannot do: the call
    returns PSWFE_E_ARG before it enqueues anything, and the capture (which holds other work)
    ends normally and replays."""
    x, q, L = W.uniform_pm1(400, seed=66)
    c = pw.choose_params(1e-6, L, m=16)
    plan = pw.Plan(c, "fp32", n_max=len(q))
    X, Q = tdev(x, torch.float32), tdev(q, torch.float32)
    plan.compute(X, Q)
    counter = torch.zeros(1, device=dev())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    status = None
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            counter.add_(1.0)
            try:
                plan.compute(X, Q, check=True)
            except pw.PswfeError as e:
                status = e.status
    assert status == pw.E_ARG
    g.replay()
    g.replay()
    torch.cuda.synchronize()
    assert float(counter[0]) == 2.0
