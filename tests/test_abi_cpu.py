"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/fem.h declares, fills the parameter struct with the
documented defaults, and rejects malformed problems with FEM_E_INVAL /
FEM_E_UNSUPPORTED before touching a device."""
import os
import re

import numpy as np
import pytest

from paper_2412_09285_amd import fem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "fem.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = fem.lib()
    names = declared_functions()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding covers all of them
    assert set(names) <= set(fem._SIGS), set(names) - set(fem._SIGS)


def test_noalloc_scratch_size_matches_header():
    txt = open(os.path.join(ROOT, "include", "fem.h")).read()
    m = re.search(r"#define FEM_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", txt)
    assert m and int(m.group(1)) << int(m.group(2)) == fem.NOALLOC_SCRATCH_BYTES


def test_abi_version_and_status_strings():
    assert fem.lib().fem_abi_version() == 2
    assert fem.status_str(0) == "FEM_OK"
    assert fem.status_str(-1) == "FEM_E_INVAL"
    assert fem.status_str(-6) == "FEM_E_UNSUPPORTED"


def test_params_default_layout():
    p = fem.default_params()
    assert (p.replicas, p.steps, p.schedule) == (16, 500, 0)
    assert (p.beta_min, p.beta_max, p.lr) == (0.01, 5.0, 0.1)
    assert (p.adam_b1, p.adam_b2, p.adam_eps, p.weight_decay) == (0.9, 0.999, 1e-8, 0.0)
    assert (p.lam, p.lambda_ramp, p.marginal_dtype) == (0.0, 0, 0)
    assert (p.energy_every, p.record_energies, p.eval_every, p.keep_grad) == (1, 0, 0, 0)
    assert (p.optimizer, p.momentum, p.rms_alpha, p.dampening) == (0, 0.0, 0.99, 0.0)


@pytest.mark.parametrize("args,msg", [
    ((3, [0], [0], None), "self-loop"),
    ((3, [0, 1], [1, 0], None), "duplicate edge"),
    ((3, [0], [5], None), "out of range"),
    ((0, [], [], None), "n must be >= 1"),
    ((3, [0], [1], [np.inf]), "not finite"),
])
def test_maxcut_rejects_malformed(args, msg):
    with pytest.raises(fem.FemError) as ei:
        fem.Problem.maxcut(*args)
    assert ei.value.status == fem.FEM_E_INVAL and msg in ei.value.message


def test_bmincut_rejects():
    with pytest.raises(fem.FemError) as ei:
        fem.Problem.bmincut(3, [0], [1], None, 1)
    assert ei.value.status == fem.FEM_E_INVAL
    with pytest.raises(fem.FemError) as ei:
        fem.Problem.bmincut(3, [0], [1], None, 3)
    assert ei.value.status == fem.FEM_E_UNSUPPORTED
    with pytest.raises(fem.FemError) as ei:
        fem.Problem.bmincut(3, [0], [1], [-1.0], 4)
    assert ei.value.status == fem.FEM_E_INVAL and "> 0" in ei.value.message
    # unit weights: the column sums and squared group sizes are exact up to
    # 2^22 nodes per instance (the bound weighted problems have on sum V_i)
    with pytest.raises(fem.FemError) as ei:
        fem.Problem.bmincut((1 << 22) + 1, [0], [1], None, 4)
    assert ei.value.status == fem.FEM_E_UNSUPPORTED and "2^22" in ei.value.message


@pytest.mark.parametrize("n,off,lits,status,msg", [
    (3, [0, 0], [], fem.FEM_E_INVAL, "empty"),
    (3, [0, 2], [1, 0], fem.FEM_E_INVAL, "out of range"),
    (3, [0, 2], [1, -4], fem.FEM_E_INVAL, "out of range"),
    (3, [0, 2, 1], [1, 2], fem.FEM_E_INVAL, "nondecreasing"),
    (6, [0, 5], [1, 2, 3, 4, 5], fem.FEM_E_UNSUPPORTED, "more than 4"),
])
def test_maxsat_rejects(n, off, lits, status, msg):
    with pytest.raises(fem.FemError) as ei:
        fem.Problem.maxsat(n, off, lits)
    assert ei.value.status == status and msg in ei.value.message


def test_valid_problem_without_device_reports_hip_error():
    """On a host without a GPU a valid problem fails at the device check with
    FEM_E_HIP (never silently on the CPU)."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(fem.FemError) as ei:
        fem.Problem.maxcut(3, [0], [1])
    assert ei.value.status == fem.FEM_E_HIP
