"""The C example program, which uses the library through its C ABI alone
(no Python, no torch), against the Python binding and the oracle: the 6^3
cube load run in 5 increments with the adaptive inner tolerance."""
import os
import subprocess

import numpy as np
import pytest

import synth
from oracle import fe, newton

pytestmark = pytest.mark.gpu


def _write_problem(prob, path, lattice=False):
    with open(path, "wb") as f:
        np.array([prob.n_nodes, prob.n_tets, len(prob.tris)], np.int64).tofile(f)
        np.ascontiguousarray(prob.X, np.float64).tofile(f)
        np.ascontiguousarray(prob.tets, np.int32).tofile(f)
        np.ascontiguousarray(prob.mat_id, np.int32).tofile(f)
        np.ascontiguousarray(prob.dir_mask, np.uint8).tofile(f)
        np.ascontiguousarray(prob.tris, np.int32).reshape(-1, 3).tofile(f)
        np.ascontiguousarray(prob.traction, np.float64).reshape(-1, 3).tofile(f)
        np.array([len(prob.materials)], np.int32).tofile(f)
        for m in prob.materials:
            np.array([m["model"]], np.int32).tofile(f)
            np.array([m["c10"], m.get("c01", 0.0), m["kappa"], m.get("k1", 0.0), m.get("k2", 0.0)],
                     np.float64).tofile(f)
        if lattice:
            np.array([1], np.int32).tofile(f)
            np.ascontiguousarray(prob.lattice, np.int32).tofile(f)


def test_c_driver_load_run(lib, tmp_path):
    import torch
    from paper_1312_5561_amd import build as b
    if not os.path.exists(b.DRIVER):
        raise RuntimeError(f"{b.DRIVER} is missing: run the build first")
    prob = synth.cube_problem(6)
    problem, state = str(tmp_path / "cube6.bin"), str(tmp_path / "state.bin")
    _write_problem(prob, problem)
    print("[c driver] cube6 5 increments adaptive", flush=True)
    r = subprocess.run([b.DRIVER, problem, "5", state, "1"], capture_output=True, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stderr
    assert r.stdout.count("converged 1") == 5
    v = np.fromfile(state, np.float64)
    assert v.shape == (4 * prob.n_nodes,)
    ctx = lib.Context(0)
    ctx.set_problem(prob)
    vt = torch.zeros(4 * prob.n_nodes, dtype=torch.float64, device="cuda")
    for k in range(1, 6):
        info, code = ctx.newton_solve(vt, k / 5.0, lib.newton_solve_params(adaptive=1))
        assert code == 0
    vp = vt.cpu().numpy()
    assert np.linalg.norm(v - vp) <= 1e-12 * np.linalg.norm(vp)
    disc = fe.Discretization(prob)
    vo = newton.load_run(disc, 5, newton.NewtonParams(adaptive=True))
    assert np.linalg.norm(v - vo) <= 1e-9 * np.linalg.norm(vo)


def test_c_driver_learned_weights(lib, tmp_path):
    """The C program with the committed raw weight file (hfsi_mlp_load) and
    the lattice coordinates: learned interpolation under the classical judge
    with the fp32 cycle, the same states as the Python binding with the
    weights set from the training checkpoint, and the oracle's to 1e-9."""
    import torch
    from paper_1312_5561_amd import build as b
    from paper_1312_5561_amd import train_mlp
    prob = synth.cube_problem(6, jitter=0.1, seed=4)
    problem, state = str(tmp_path / "cube6l.bin"), str(tmp_path / "state.bin")
    _write_problem(prob, problem, lattice=True)
    print("[c driver] cube6 learned weights, 3 increments", flush=True)
    r = subprocess.run([b.DRIVER, problem, "3", state, "0", train_mlp.DEFAULT_RAW_WEIGHTS], capture_output=True,
                       text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stderr
    v = np.fromfile(state, np.float64)
    ctx = lib.Context(0)
    ctx.set_problem(prob)
    w, _ = train_mlp.load(train_mlp.DEFAULT_WEIGHTS)
    ctx.mlp_set_weights(w)
    prm = lib.newton_solve_params(step=lib.newton_params(
        amg=lib.amg_params(precision=1, interp=1), solve=lib.solve_params()))
    vt = torch.zeros(4 * prob.n_nodes, dtype=torch.float64, device="cuda")
    for k in range(1, 4):
        info, code = ctx.newton_solve(vt, k / 3.0, prm)
        assert code == 0
    vp = vt.cpu().numpy()
    assert np.linalg.norm(v - vp) <= 1e-12 * np.linalg.norm(vp)
    vo = newton.load_run(fe.Discretization(prob), 3, newton.NewtonParams())
    assert np.linalg.norm(v - vo) <= 1e-9 * np.linalg.norm(vo)
    # without lattice coordinates the program refuses the weight file
    _write_problem(prob, problem, lattice=False)
    r = subprocess.run([b.DRIVER, problem, "3", state, "0", train_mlp.DEFAULT_RAW_WEIGHTS], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2


@pytest.mark.parametrize("variant", ["coupled", "additive"])
def test_c_driver_coupled_vanka(lib, tmp_path, variant):
    """The C program with the coupled displacement-pressure AMG and the
    multiplicative Vanka smoother (amg params coupled = 1) or its additive
    variant (coupled = 2) as the preconditioner: the load run reaches the
    oracle's converged states."""
    from paper_1312_5561_amd import build as b
    prob = synth.cube_problem(6, jitter=0.1, seed=4)
    problem, state = str(tmp_path / "cube6v.bin"), str(tmp_path / "state.bin")
    _write_problem(prob, problem, lattice=False)
    print(f"[c driver] cube6 {variant} Vanka AMG, 3 increments", flush=True)
    r = subprocess.run([b.DRIVER, problem, "3", state, "0", variant], capture_output=True, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stderr
    v = np.fromfile(state, np.float64)
    vo = newton.load_run(fe.Discretization(prob), 3, newton.NewtonParams())
    assert np.linalg.norm(v - vo) <= 1e-9 * np.linalg.norm(vo)
