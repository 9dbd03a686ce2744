"""The C-ABI library loads on the CPU host and exports every function that
include/irlnqs.h declares (no device calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "irlnqs.h")
LIB = os.path.join(ROOT, "paper_2601_01437_amd", "lib", "libirlnqs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(irl_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("irl_system_create", "irl_nqs_evaluate", "irl_apply_lm_operator",
                     "irl_step", "irl_dtilde_set", "irl_debug_excitations"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2601_01437_amd import binding
    assert sorted(binding.EXPORTED) == declared_functions()


def _c_sizes():
    """sizeof of the ABI structs as the C compiler lays them out."""
    import subprocess
    import tempfile
    names = ["irl_system_desc", "irl_system_info", "irl_nqs_desc", "irl_eval_out",
             "irl_solver_opts", "irl_step_result", "irl_adam_opts", "irl_vmc_out"]
    body = "".join(f'printf("%zu\\n", sizeof({n}));' for n in names)
    src = f'#include <stdio.h>\n#include "irlnqs.h"\nint main(void){{{body}return 0;}}\n'
    with tempfile.TemporaryDirectory() as d:
        p, exe = os.path.join(d, "t.c"), os.path.join(d, "t")
        open(p, "w").write(src)
        r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                            p, "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    return dict(zip(names, map(int, out)))


def test_struct_layout_matches_c_compiler():
    from paper_2601_01437_amd import binding as B
    sizes = _c_sizes()
    for name, size in sizes.items():
        assert ctypes.sizeof(getattr(B, name)) == size, name


def test_enum_values_match_header():
    """Every IRL_* enumerator the header defines has the same value in the binding."""
    from paper_2601_01437_amd import binding
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    values = {}
    for body in re.findall(r"enum\s+\w+\s*\{(.*?)\}", text, flags=re.S):
        for name, val in re.findall(r"\b(IRL_[A-Z0-9_]+)\s*=\s*(-?\d+)u?", body):
            values[name] = int(val)
    assert values["IRL_MODE_C"] == 2
    # the statistics kinds are the binding's STAT_KINDS, in enum order (the
    # binding spells the reduced-precision kinds _LO as _fp32)
    stats = {n: v for n, v in values.items() if n.startswith("IRL_STAT_")}
    for n in stats:
        del values[n]
    assert stats.pop("IRL_STAT_KINDS") == len(binding.STAT_KINDS)
    assert {n[len("IRL_STAT_"):].lower().replace("_lo", "_fp32"): v for n, v in stats.items()} == \
        {k: i for i, k in enumerate(binding.STAT_KINDS)}
    missing = [n for n in values if not hasattr(binding, n)]
    assert not missing, missing
    wrong = {n: (v, getattr(binding, n)) for n, v in values.items() if getattr(binding, n) != v}
    assert not wrong, wrong
