"""The C ABI library loads and exports every entry point include/mpt.h
declares (CPU only: no call that needs a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mpt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpt_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mpt_scene_upload", "mpt_solve_batch", "mpt_accept", "mpt_create", "mpt_destroy",
                 "mpt_mlp_train_step", "mpt_mlp_predict"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2301_06399_amd import mpt
    if not os.path.exists(mpt.LIB_PATH):
        from paper_2301_06399_amd.build import build
        build()
    lib = C.CDLL(mpt.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(mpt.EXPORTS) == declared_functions()


def test_default_options_are_host_only():
    from paper_2301_06399_amd import mpt
    o = mpt.default_opts()
    assert o.precision == mpt.FP32_POLISH64 and o.max_iter == 200 and o.plateau_win == 10
    assert o.tau_root == 1e-9 and o.tol_step == 1e-12 and o.polish_gate == 1e-2
    with pytest.raises(KeyError):
        mpt.default_opts(no_such_option=1)


def test_oracle_library_is_independent_of_the_hip_library():
    """The oracle shares no code with the HIP path: no include, no import."""
    hip_dir = os.path.join(ROOT, "paper_2301_06399_amd")
    for dp, _, fs in os.walk(hip_dir):
        for f in fs:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                t = open(os.path.join(dp, f)).read()
                assert not re.search(r"(import\s+oracle|from\s+oracle|mpt_oracle|orc_)", t), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".c", ".h", ".py")):
            t = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2301_06399_amd" not in t and "mpt_device" not in t, f


def test_bit_rows_unpack_like_the_header_says():
    """Bit j of a row of W words is word j / 32, bit j % 32 (the layout of
    the visibility matrix, BS row and UE columns)."""
    import numpy as np
    from paper_2301_06399_amd import mpt
    rng = np.random.default_rng(3)
    n = 77
    bits = rng.random((5, n)) < 0.3
    W = (n + 31) // 32
    words = np.zeros((5, W), np.uint32)
    for r in range(5):
        for j in np.where(bits[r])[0]:
            words[r, j // 32] |= np.uint32(1) << np.uint32(j % 32)
    assert np.array_equal(mpt.unpack_bits(words.view(np.int32), n), bits)
    assert np.array_equal(mpt.unpack_bits(words[0].view(np.int32), n), bits[0])


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every field of the binding's ctypes structs sits at the offset and
    has the size the C compiler gives it in include/mpt.h, and each struct
    has the C size: the binding and the library read the same bytes."""
    import subprocess
    from paper_2301_06399_amd import mpt
    structs = {"mpt_scene_desc": mpt.SceneDesc, "mpt_batch_desc": mpt.BatchDesc,
               "mpt_solve_opts": mpt.SolveOpts, "mpt_solve_out": mpt.SolveOut}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mpt.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu %zu\\n", offsetof({cname}, {fname}), '
                         f'sizeof((({cname} *)0)->{fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        parts = line.split()
        if len(parts) == 3 and parts[1] == "size":
            got[(parts[0], None)] = int(parts[2])
        elif len(parts) == 4:
            got[(parts[0], parts[1])] = (int(parts[2]), int(parts[3]))
    for cname, py in structs.items():
        assert got[(cname, None)] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            f = getattr(py, fname)
            assert got[(cname, fname)] == (f.offset, f.size), (cname, fname)


def test_assembly_flops_are_a_proper_part_of_an_iteration():
    """The assembly count is positive and below a whole LM iteration for every
    order and type sequence, in both forms (host-only calls)."""
    from paper_2301_06399_amd import mpt
    for form in (mpt.FORM_IMPLICIT, mpt.FORM_PARAMETRIC):
        tab = mpt.flops_table(form)
        for n in range(1, 6):
            a, lm = tab[n]["assembly"], tab[n]["lm"]
            assert (a > 0).all() and (a < lm).all(), (form, n)
    with pytest.raises(mpt.MptError):
        mpt.flops_per_iter([0, 7], mpt.FORM_IMPLICIT)


def test_bench_flop_count_bounds_kept_iterations():
    """The roofline's FLOP count charges the FP32 orders 1-3 iterations after
    a path's first without their assembly (a lower bound) and charges orders
    4-5 and the uncorrected count in full."""
    import importlib.util
    import numpy as np
    from paper_2301_06399_amd import mpt
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    tab = mpt.flops_table(mpt.FORM_PARAMETRIC)
    order = np.array([3, 3, 4, 5, 3], np.int32)
    code = np.array([0, 1 + 4 * 2, 5, 21, 2], np.int64)
    iters = np.array([1, 7, 9, 4, 0], np.int32)
    full = bench.algorithmic_flops(tab, order, code, iters, "lm")
    low = bench.algorithmic_flops(tab, order, code, iters, "lm", kept=True)
    want_full = sum(int(tab[n]["lm"][c]) * int(i) for n, c, i in zip(order, code, iters))
    skipped = int(tab[3]["assembly"][1 + 4 * 2]) * 6     # the 7-iteration order-3 path
    assert full == want_full and low == full - skipped
