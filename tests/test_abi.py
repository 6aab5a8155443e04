"""The C-ABI library loads on a machine without a GPU and exports every entry
point that include/craneplan.h declares (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "craneplan.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cp_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("cp_plan_create", "cp_eval_paths", "cp_eval_paths_backward", "cp_optimizer_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2503_14160_amd import craneplan
    if not os.path.exists(craneplan.LIB_PATH):
        from paper_2503_14160_amd import build
        build.build()
    L = ctypes.CDLL(craneplan.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(craneplan.EXPORTS) == _declared()


def test_binding_raises_when_library_missing(monkeypatch, tmp_path):
    from paper_2503_14160_amd import craneplan
    monkeypatch.setattr(craneplan, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(craneplan, "_lib", None)
    with pytest.raises(ImportError):
        craneplan.lib()


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2503_14160_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "oracle.c" not in txt, f


def test_batch_rejects_polish_before_touching_the_device():
    """Argument checks run before any device work (no GPU needed)."""
    import numpy as np

    from paper_2503_14160_amd import craneplan, synth
    p = synth.c0_plain()
    p.opt = synth.OptParams(B=16, nu=2, sigma0=0.2, eps=1e-6, seed=1, T=1, polish_elites=2, polish_steps=3)
    with pytest.raises(craneplan.CranePlanError) as ei:
        craneplan.Batch([p])
    assert ei.value.code == -1


def test_plan_argument_errors_without_device():
    import numpy as np

    from paper_2503_14160_amd import craneplan, synth
    p = synth.c0_plain()
    bad = synth.CostParams(K=0, M=16)
    with pytest.raises(craneplan.CranePlanError) as ei:
        craneplan.Plan(p.robot, p.scene, bad, max_B=4)
    assert ei.value.code == -2
    smooth0 = synth.CostParams(K=4, M=4, hinge=synth.HINGE_SMOOTH, margin=0.0)
    with pytest.raises(craneplan.CranePlanError) as ei:
        craneplan.Plan(p.robot, p.scene, smooth0, max_B=4)
    assert ei.value.code == -1
    rb = synth.make_robot(3, 8)
    rb.axis = rb.axis * 2.0
    with pytest.raises(craneplan.CranePlanError) as ei:
        craneplan.Plan(rb, p.scene, p.cost, max_B=4)
    assert "unit" in str(ei.value)
    for mode in (-1, 4):
        with pytest.raises(craneplan.CranePlanError) as ei:
            craneplan.Plan(p.robot, p.scene, p.cost, max_B=4, pair_filter=mode)
        assert "pair_filter" in str(ei.value)


def test_tune_rejects_no_target_before_touching_the_device():
    from paper_2503_14160_amd import craneplan
    if not os.path.exists(craneplan.LIB_PATH):
        from paper_2503_14160_amd import build
        build.build()
    with pytest.raises(craneplan.CranePlanError):
        craneplan.tune()


def test_sdf_build_argument_checks_without_device():
    """cp_sdf_build refuses grid sizes outside 2..4096 per axis (the distance
    transforms' per-line stacks are sized for that) and other bad arguments
    before any device work."""
    import ctypes

    import numpy as np

    from paper_2503_14160_amd import craneplan
    if not os.path.exists(craneplan.LIB_PATH):
        from paper_2503_14160_amd import build
        build.build()
    L = craneplan.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the checks fail first
    org = np.zeros(3, np.float32)
    for dims, voxel, code in (((4097, 4, 4), 0.1, -2), ((4, 1, 4), 0.1, -2), ((8, 8, 8), 0.0, -1),
                              ((8, 8, 8), float("nan"), -1)):
        d = np.array(dims, np.int32)
        rc = L.cp_sdf_build(fake, 10, d.ctypes.data, org.ctypes.data, voxel, fake, None, None, None, None)
        assert rc == code, (dims, voxel, rc)
    d = np.array((8, 8, 8), np.int32)
    assert L.cp_sdf_build(fake, -1, d.ctypes.data, org.ctypes.data, 0.1, fake, None, None, None, None) == -2
    assert L.cp_sdf_build(None, 10, d.ctypes.data, org.ctypes.data, 0.1, fake, None, None, None, None) == -1


def test_ik_argument_checks_without_device():
    """cp_ik_solve / cp_debug_ik_residual refuse bad weights, iteration
    limits, sizes and a best-row output without the per-row costs before
    touching the plan or the device."""
    import ctypes

    from paper_2503_14160_amd import craneplan, synth
    if not os.path.exists(craneplan.LIB_PATH):
        from paper_2503_14160_amd import build
        build.build()
    L = craneplan.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the checks fail first

    def solve(par, N=8, restarts=1, info=fake, best=None, plan=fake):
        k = craneplan._Ik()
        craneplan._fill_ik(k, par)
        return L.cp_ik_solve(plan, ctypes.byref(k), fake, fake, None, N, restarts, fake, info, None, best, None)

    good = synth.IkParams()
    assert solve(good, plan=None) == -1
    for bad in (dict(lambda_q=-1.0), dict(lambda_c=float("nan")), dict(max_iters=-1), dict(max_iters=1001),
                dict(tau=0.0), dict(eps_grad=-1e-3), dict(eps_step=float("inf"))):
        par = synth.IkParams(**bad)
        assert solve(par) == -1, bad
    assert solve(good, N=0) == -2
    assert solve(good, N=(1 << 20) + 1) == -2
    assert solve(good, N=10, restarts=4) == -2
    assert solve(good, N=8, restarts=0) == -2
    assert solve(good, N=8, restarts=4, info=None, best=fake) == -1
    k = craneplan._Ik()
    craneplan._fill_ik(k, synth.IkParams(lambda_r=-1.0))
    assert L.cp_debug_ik_residual(fake, ctypes.byref(k), fake, fake, None, 4, fake, fake, None) == -1
