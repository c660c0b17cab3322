"""Parity at the workloads' full sizes, in the launch configuration bench.py times.

128^3 / 128 angles: Algorithm 8 for 100 iterations with the 20-step power
iteration, FP32 (FP64 reductions) and all-FP64, against the oracle's
iterate at 4096 sampled voxels, its objective history and step size.
256^3 / 256 angles: forward and adjoint at 4096 sampled outputs, the autograd
gradient A^T (A h - d) on the central 16^3 crop, and central finite
differences on 16 random directions (a property that holds at any size).
Expected values: tests/golden/*_oracle.json, written by
tests/golden/make_golden.py from the oracle alone.
"""
import json
import os

import numpy as np
import pytest

from conftest import rel_l2, to_dev, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def _load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated")
    return json.load(open(path))


def _golden_mod():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def c256():
    import synth
    gold = _load("c256_oracle.json")
    mg = _golden_mod()
    case = mg.as_f32_values(synth.make_case("c256", gold["seed"]))
    data = synth.random_field((len(case.angles), case.n, case.n), gold["data_seed"])
    data = data.astype(np.float32).astype(np.float64)
    return gold, case, data


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_c256_forward_adjoint_samples(c256, dtype):
    import paper_1901_06503_amd as ff
    gold, case, data = c256
    print(f"[fullsize] 256^3 forward/adjoint {dtype}", flush=True)
    with ff.Plan(to_dev(case.c, dtype), case.dx, case.T, case.angles) as P:
        # the benchmark's kernels: two steps per pass; on 256 compute units the FP32
        # plan takes 128 x 16 tiles (pairs of x-adjacent points per lane), FP64 64 x 16,
        # one z-chunk round each
        assert P.steps_per_pass == 2
        if torch.cuda.get_device_properties(0).multi_processor_count == 256:
            assert P.stencil_shape == ((128, 16, 32) if dtype == torch.float32 else (64, 16, 64))
        fwd = P.forward(to_dev(case.h_true, dtype)).double().flatten()
        fi = torch.tensor(gold["forward_index"], device="cuda")
        got = fwd[fi].cpu().numpy()
        adj = P.adjoint(to_dev(data, dtype)).double().flatten()
        ai = torch.tensor(gold["adjoint_index"], device="cuda")
        got_a = adj[ai].cpu().numpy()
        tol = 1e-5 if dtype == torch.float32 else 1e-12
        assert rel_l2(got, np.array(gold["forward_sample"])) <= tol
        assert rel_l2(got_a, np.array(gold["adjoint_sample"])) <= tol
        assert abs(float(fwd.norm()) / gold["forward_norm"] - 1) <= tol
        assert abs(float(adj.norm()) / gold["adjoint_norm"] - 1) <= tol


def test_c256_autograd_gradient_crop_and_fd(c256):
    import paper_1901_06503_amd as ff
    from paper_1901_06503_amd.autograd import xw
    from test_gpu_autograd import _fd_check
    gold, case, data = c256
    print("[fullsize] 256^3 autograd", flush=True)
    with ff.Plan(to_dev(case.c, torch.float32), case.dx, case.T, case.angles) as P:
        h = to_dev(case.h_true, torch.float32).requires_grad_(True)
        d = to_dev(data, torch.float32)
        loss = 0.5 * torch.sum((xw(P, h) - d) ** 2)
        loss.backward()
        c0, m = gold["crop_origin"], gold["crop_size"]
        crop = to_np(h.grad[c0:c0 + m, c0:c0 + m, c0:c0 + m]).ravel()
        assert rel_l2(crop, np.array(gold["gradient_crop"])) <= 1e-4
        assert abs(float(h.grad.double().norm()) / gold["gradient_norm"] - 1) <= 1e-5
        assert _fd_check(P, h.detach(), d, 16, 1e-3, 11) <= 1e-3


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_c384_full_size_adjoint_dot_test(dtype):
    """384^3 / 360 angles / T = 0.6 at full size, in the kernels the plan picks (two
    leapfrog steps per pass, staged X and X^T): <A h, g> = <h, A^T g> for random h
    and g (a property of the exact discrete transpose that holds at any size)."""
    import paper_1901_06503_amd as ff
    import synth
    case = synth.make_case("c384", 4001)
    print(f"[fullsize] 384^3 dot test {dtype}", flush=True)
    gen = torch.Generator(device="cuda").manual_seed(7)
    with ff.Plan(to_dev(case.c, dtype), case.dx, case.T, case.angles) as P:
        assert P.steps_per_pass == 2
        h = torch.randn(P.shape, dtype=dtype, device="cuda", generator=gen)
        g = torch.randn(P.data_shape, dtype=dtype, device="cuda", generator=gen)
        Ah = P.forward(h)
        ATg = P.adjoint(g)
        lhs = float(torch.dot(Ah.double().flatten(), g.double().flatten()))
        rhs = float(torch.dot(h.double().flatten(), ATg.double().flatten()))
        scale = float(Ah.double().norm() * g.double().norm())
    tol = 1e-12 if dtype == torch.float64 else 2e-5
    assert abs(lhs - rhs) <= tol * scale


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_c48_reconstruction_end_to_end(oracle, dtype):
    """48^3 / 48 angles / T = 0.5 / 1% noise / 5 iterations of Algorithm 8 with the
    20-step power iteration: data simulation, step size and iterates by the oracle,
    live (a second or two on the host), against the GPU in FP64 and FP32."""
    import time
    import paper_1901_06503_amd as ff
    import synth
    mg = _golden_mod()
    case = mg.as_f32_values(synth.make_case("c48_f64", 1001))
    g = mg.geometry(case)
    t0 = time.perf_counter()
    G = mg.simulate(case, g)
    h_ref, obj_ref, s_ref = oracle.fb(g, case.c, G, case.lam, step=0.0, n_iter=case.n_iter, n_power=case.n_power,
                                      flags=oracle.POSITIVITY | oracle.PRECOND)
    print(f"[fullsize] 48^3 oracle end to end {time.perf_counter() - t0:.2f} s, {dtype}", flush=True)
    with ff.Plan(to_dev(case.c, dtype), case.dx, case.T, case.angles) as P:
        assert P.nt == oracle.plan_info(g, case.c)[0]
        res = P.reconstruct(to_dev(G, dtype), case.lam, case.n_iter, step=0.0, n_power=case.n_power)
    tol = 1e-10 if dtype == torch.float64 else 1e-4
    assert res.step == pytest.approx(s_ref, rel=tol)
    assert rel_l2(to_np(res.h), h_ref) <= tol
    assert np.allclose(res.objective, obj_ref, rtol=tol, atol=0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_c128_reconstruction_100_iterations(oracle, dtype):
    import paper_1901_06503_amd as ff
    import synth
    gold = _load("c128_oracle.json")
    mg = _golden_mod()
    case = mg.as_f32_values(synth.make_case("c128", gold["seed"]))
    g = mg.geometry(case)
    G = mg.simulate(case, g)                   # oracle data simulation (same as the fixture's)
    print(f"[fullsize] 128^3 reconstruction {dtype}", flush=True)
    with ff.Plan(to_dev(case.c, dtype), case.dx, case.T, case.angles) as P:
        res = P.reconstruct(to_dev(G, dtype), gold["lam"], gold["n_iter"], step=0.0, n_power=gold["n_power"])
        idx = torch.tensor(gold["sample_index"], device="cuda")
        got = res.h.double().flatten()[idx].cpu().numpy()
    tol = 1e-4 if dtype == torch.float32 else 1e-10
    assert res.step == pytest.approx(gold["step"], rel=tol)
    assert rel_l2(got, np.array(gold["h_sample"])) <= tol
    assert np.allclose(res.objective, gold["objective"], rtol=tol, atol=0)
    assert abs(float(res.h.double().norm()) / gold["h_norm"] - 1) <= tol


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_c384_window_reconstruction_200_iterations(oracle, dtype):
    """Precision study: the central 64^3 window of the 384^3 workload (dx = 3/383,
    T = 0.6, 360 angles) as a standalone problem, 200 iterations, against the oracle;
    FP32 fields with FP64 reductions and all-FP64."""
    import paper_1901_06503_amd as ff
    import synth
    gold = _load("c384crop_oracle.json")
    mg = _golden_mod()
    case = mg.as_f32_values(synth.make_case("c384", gold["seed"], n=64, dx=synth.grid_spacing(384)))
    g = mg.geometry(case)
    G = mg.simulate(case, g)
    print(f"[fullsize] 384^3 window, 200 iterations, {dtype}", flush=True)
    with ff.Plan(to_dev(case.c, dtype), case.dx, case.T, case.angles) as P:
        res = P.reconstruct(to_dev(G, dtype), gold["lam"], gold["n_iter"], step=0.0, n_power=gold["n_power"])
        idx = torch.tensor(gold["sample_index"], device="cuda")
        got = res.h.double().flatten()[idx].cpu().numpy()
        norm = float(res.h.double().norm())
    tol = 1e-4 if dtype == torch.float32 else 1e-10
    assert res.step == pytest.approx(gold["step"], rel=tol)
    assert rel_l2(got, np.array(gold["h_sample"])) <= tol
    assert np.allclose(res.objective, gold["objective"], rtol=tol, atol=0)
    assert abs(norm / gold["h_norm"] - 1) <= tol
