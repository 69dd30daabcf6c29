"""The C-ABI library loads and exports every symbol include/vmcdet.h declares
(no compute: CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "vmcdet.h")) as f:
        txt = f.read()
    return sorted(set(re.findall(r"^\s*(?:vmc_status|const char\*)\s+(vmc_\w+)\(", txt, re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ["vmc_create", "vmc_build_slater", "vmc_ilutp", "vmc_det_ratio", "vmc_accept",
                 "vmc_run_sweeps", "vmc_run_steps", "vmc_destroy"]:
        assert must in names


def test_library_exports_all_symbols():
    from paper_1008_5113_amd.vmcdet import EXPORTED, LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(EXPORTED) == _declared()


def test_struct_layouts_match_header():
    import subprocess
    import tempfile
    from paper_1008_5113_amd import vmcdet as v
    src = ('#include <stdio.h>\n#include "vmcdet.h"\nint main(){printf("%zu %zu %zu %zu %zu",'
           'sizeof(vmc_params),sizeof(vmc_walker_init),sizeof(vmc_stats),sizeof(vmc_state_view),'
           'sizeof(vmc_step_record));return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        with open(c, "w") as f:
            f.write(src)
        subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    sizes = [ctypes.sizeof(t) for t in (v.VmcParams, v.VmcWalkerInit, v.VmcStats, v.VmcStateView,
                                        v.VmcStepRecord)]
    assert [int(x) for x in out] == sizes


def test_default_params_without_gpu():
    from paper_1008_5113_amd.vmcdet import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("library not built")
    import paper_1008_5113_amd as vm
    p = vm.default_params()
    assert p.gmres_maxit == 40 and p.droptol == 1e-4 and p.permtol == 0.1 and p.n_thresh == 100.0


def test_binding_rejects_mismatched_arrays_before_the_library():
    """The binding checks the array shapes the library will copy from (n*3
    sites, n widths, n*3 positions) and raises before any device call."""
    from paper_1008_5113_amd.vmcdet import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("library not built")
    import numpy as np
    import paper_1008_5113_amd as vm
    import workloads as wl
    inst = wl.small_instance((2, 2, 2))
    s = inst.systems[0]
    good = inst.walkers[0].pos0
    for bad in (good[:-1], good[:, :2], good.reshape(-1)):
        with pytest.raises(ValueError):
            vm.Context([s], [(0, bad, 0)], vm.default_params())
    s2 = wl.make_system((2, 2, 2))
    s2.sigma = np.full(s2.sigma.shape[0] - 1, 0.35)
    with pytest.raises(ValueError):
        vm.Context([s2], [(0, good, 0)], vm.default_params())


def test_binding_constants_match_header():
    """Status codes, precisions and step-record flags of the binding are the
    header's #define values."""
    from paper_1008_5113_amd import vmcdet as v
    with open(os.path.join(ROOT, "include", "vmcdet.h")) as f:
        defs = dict(re.findall(r"^#define\s+(VMC_\w+)\s+\(?(-?\d+)\)?", f.read(), re.M))
    names = {k: k for k in ("VMC_OK", "VMC_EINVAL", "VMC_ENOMEM", "VMC_EHIP", "VMC_ENOCONV",
                            "VMC_ESINGULAR", "VMC_ECAPACITY", "VMC_ESTATE")}
    names.update({"PREC_FP64": "VMC_PREC_FP64", "PREC_MIXED": "VMC_PREC_MIXED"})
    names.update({f"FLAG_{k}": f"VMC_FLAG_{k}" for k in ("ACCEPTED", "REORDERED", "REFACTORED",
                                                         "CONVERGED", "SINGULAR", "CAPACITY", "TRIG_N",
                                                         "TRIG_NOCONV", "TRIG_ITERS", "TRIG_FORCED",
                                                         "NOCONV")})
    for py, c in names.items():
        assert getattr(v, py) == int(defs[c]), (py, c)


def test_missing_library_fails_loudly(tmp_path):
    """No fallback: loading a library that is not there raises ImportError."""
    from paper_1008_5113_amd import vmcdet as v
    with pytest.raises(ImportError):
        v.load_library(str(tmp_path / "libvmcdet.so"))
