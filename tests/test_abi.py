"""The C-ABI library loads and exports every entry point include/mpm.h
declares, and the ctypes structures match the C layout (no GPU needed)."""
import ctypes
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mpm_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("mpm_sparse_build", "mpm_p2g", "mpm_grid_update", "mpm_g2p", "mpm_step",
                     "mpm_create", "mpm_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2605_28525_amd import mpm as M
    lib = ctypes.CDLL(M._LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert M.lib.mpm_status_string(4).startswith(b"MPM_ERR_OVERFLOW")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_struct_layout_matches_c():
    from paper_2605_28525_amd import mpm as M
    structs = (M.mpm_params, M.mpm_particles, M.mpm_instance)
    body = []
    for st in structs:
        body.append(f'printf("sizeof.{st.__name__} %zu\\n", sizeof({st.__name__}));')
        body += [f'printf("{st.__name__}.{f} %zu\\n", offsetof({st.__name__}, {f}));' for f, _ in st._fields_]
    src = "#include <stdio.h>\n#include <stddef.h>\n#include \"mpm.h\"\nint main(void) {\n" + \
        "\n".join(body) + "\nreturn 0;\n}\n"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.strip().splitlines():
        k, v = line.split()
        got[k] = int(v)
    for struct in structs:
        assert got[f"sizeof.{struct.__name__}"] == ctypes.sizeof(struct), struct.__name__
        for name, _ in struct._fields_:
            assert got[f"{struct.__name__}.{name}"] == getattr(struct, name).offset, name


def test_constants_match_header():
    from paper_2605_28525_amd import mpm as M
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+(MPM_\w+)\s+(\d+)u?", text))
    assert int(defs["MPM_ERR_OVERFLOW"]) == M.MPM_ERR_OVERFLOW
    assert int(defs["MPM_FLAG_NAN"]) == M.MPM_FLAG_NAN
    assert int(defs["MPM_GRID_DENSE"]) == M.MPM_GRID_DENSE
    for k, v in M.MPM_BC.items():
        assert int(defs["MPM_BC_" + k.upper()]) == v
    assert int(defs["MPM_MODEL_DP"]) == M.MPM_MODEL["dp"]
    assert int(defs["MPM_MODEL_ELASTIC"]) == M.MPM_MODEL["elastic"]
    for k in ("SYNC_REBUILD", "ADJOINT", "FULL_SORT", "DETERMINISTIC_ORDER", "SCAN_BUILD"):
        assert int(defs["MPM_FLAG_" + k]) == getattr(M, "MPM_FLAG_" + k)


def test_create_rejects_bad_flag_combinations_without_touching_the_device():
    """The scan-based build is for one sparse simulation without reverse mode;
    the ascending-key order needs a sparse grid."""
    from paper_2605_28525_amd import mpm as M
    from paper_2605_28525_amd import workloads as wl
    ctx = ctypes.c_void_p()
    w = wl.tiny_3d(n=48)
    for flags, mode in ((M.MPM_FLAG_SCAN_BUILD, M.MPM_GRID_DENSE),
                        (M.MPM_FLAG_SCAN_BUILD | M.MPM_FLAG_ADJOINT, M.MPM_GRID_SPARSE),
                        (M.MPM_FLAG_DETERMINISTIC_ORDER, M.MPM_GRID_DENSE)):
        p = M.params_from_workload(w, grid_mode=mode, flags=flags)
        assert M.lib.mpm_create(ctypes.byref(p), ctypes.byref(ctx)) == M.MPM_ERR_ARG
    p = M.params_from_ensemble(wl.ensemble_small(n_instances=3), flags=M.MPM_FLAG_SCAN_BUILD)
    assert M.lib.mpm_create(ctypes.byref(p), ctypes.byref(ctx)) == M.MPM_ERR_ARG
    assert not ctx.value


def test_create_rejects_bad_arguments_without_touching_the_device():
    """Argument errors are reported before any device call."""
    from paper_2605_28525_amd import mpm as M
    p = M.mpm_params()
    p.dim = 4
    ctx = ctypes.c_void_p()
    assert M.lib.mpm_create(ctypes.byref(p), ctypes.byref(ctx)) == M.MPM_ERR_ARG
    assert not ctx.value
    assert M.lib.mpm_create(None, ctypes.byref(ctx)) == M.MPM_ERR_ARG


def test_create_rejects_bad_ensembles_without_touching_the_device():
    from paper_2605_28525_amd import mpm as M
    from paper_2605_28525_amd import workloads as wl
    ens = wl.ensemble_small(n_instances=3)
    ctx = ctypes.c_void_p()
    p = M.params_from_ensemble(ens)
    p.n_instances = 65                      # more than 64 instances
    assert M.lib.mpm_create(ctypes.byref(p), ctypes.byref(ctx)) == M.MPM_ERR_ARG
    p = M.params_from_ensemble(ens)
    p.instances = None                      # table missing
    assert M.lib.mpm_create(ctypes.byref(p), ctypes.byref(ctx)) == M.MPM_ERR_ARG
    p = M.params_from_ensemble(ens)
    p.grid_mode = M.MPM_GRID_DENSE          # dense grids have no instance bits
    assert M.lib.mpm_create(ctypes.byref(p), ctypes.byref(ctx)) == M.MPM_ERR_ARG
    p = M.params_from_ensemble(ens)
    p.flags = M.MPM_FLAG_ADJOINT
    assert M.lib.mpm_create(ctypes.byref(p), ctypes.byref(ctx)) == M.MPM_ERR_ARG
    p = M.params_from_ensemble(ens)
    p._inst_keepalive[1].dt = 0.0           # invalid instance material
    assert M.lib.mpm_create(ctypes.byref(p), ctypes.byref(ctx)) == M.MPM_ERR_ARG
    p = M.params_from_ensemble(ens)
    p.cells[0] = 1 << 20                    # instance + block + cell bits exceed 32
    assert M.lib.mpm_create(ctypes.byref(p), ctypes.byref(ctx)) == M.MPM_ERR_ARG
    assert not ctx.value
