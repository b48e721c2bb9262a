"""C-ABI checks without a GPU: the HIP library loads, exports every function that
include/zema.h declares, and the binding's ctypes structs match the header layout."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zema.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(zema_[a-z_]+)\s*\(", src)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for n in ("zema_scene_create", "zema_ip_assemble", "zema_contact_candidates", "zema_ccd_max_step",
              "zema_pcg_solve", "zema_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2311_05945_amd import zema
    L = zema.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    bound = {n for n, _ in zema.SIGNATURES}
    assert set(declared_functions()) == bound


def test_tune_knobs_match_header():
    """Every ZEMA_TUNE_* value of the header has the binding's constant of the same
    value, and no binding constant is missing from the header."""
    from paper_2311_05945_amd import zema
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    knobs = {k: int(v) for k, v in re.findall(r"\bZEMA_TUNE_([A-Z_]+)\s*=\s*(\d+)", src)}
    assert "CG_ROWS" in knobs and len(knobs) >= 6
    bound = {k[len("TUNE_"):]: getattr(zema, k) for k in dir(zema) if k.startswith("TUNE_")}
    assert bound == knobs


def test_struct_layout_matches_header(tmp_path):
    from paper_2311_05945_amd import zema
    prog = tmp_path / "sizes.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "zema.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu\\n", sizeof(zema_params), sizeof(zema_soft_desc), sizeof(zema_affine_desc),'
        " sizeof(zema_step_stats));\n"
        '  printf("%zu %zu %zu\\n", offsetof(zema_affine_desc, mode), offsetof(zema_affine_desc, kappa_A),'
        " offsetof(zema_step_stats, ms_total));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    sizes = [int(x) for x in out]
    assert sizes[:4] == [ctypes.sizeof(zema.Params), ctypes.sizeof(zema.SoftDesc), ctypes.sizeof(zema.AffineDesc),
                         ctypes.sizeof(zema.StepStats)]
    assert sizes[4:] == [zema.AffineDesc.mode.offset, zema.AffineDesc.kappa_A.offset, zema.StepStats.ms_total.offset]


def test_product_path_never_uses_the_oracle():
    pkg = os.path.join(ROOT, "paper_2311_05945_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.replace("the oracle", ""), f
                assert "zema_ref" not in txt and "zref_" not in txt, f


def test_binding_fails_loudly_without_library(monkeypatch):
    from paper_2311_05945_amd import zema
    monkeypatch.setattr(zema, "_LIB", None)
    monkeypatch.setattr(zema, "LIB_PATH", "/nonexistent/libzema.so")
    with pytest.raises(RuntimeError):
        zema.lib()


def test_argument_errors_need_no_device():
    """Entry points reject invalid arguments before any HIP call (so this runs on the
    CPU): null objects, an empty or duplicated group, unknown knobs."""
    from paper_2311_05945_amd import zema
    L = zema.lib()
    E_ARG = zema.E_ARG
    st = (ctypes.c_int32 * 2)()
    assert L.zema_step_group(None, 1, 1, None, st) == E_ARG
    one = (ctypes.c_void_p * 1)(None)
    assert L.zema_step_group(one, 0, 1, None, st) == E_ARG
    assert L.zema_step_group(one, 1, 1, None, st) == E_ARG
    v = ctypes.c_int32()
    assert L.zema_tune(None, zema.TUNE_PCG_FORM, 1) == E_ARG
    assert L.zema_tune_get(None, zema.TUNE_PCG_FORM, ctypes.byref(v)) == E_ARG
    loss = ctypes.c_double()
    buf = ctypes.c_void_p(1)
    assert L.zema_mlp_grad_noalloc(None, buf, buf, 16, buf, ctypes.byref(loss)) == E_ARG
    assert L.zema_tune(None, zema.TUNE_WARM_FIT, 2) == E_ARG
    assert L.zema_warm_fit(None, 2, buf, buf) == E_ARG


def test_noalloc_entry_point_declared_with_its_limit():
    """The allocation-free gradient is declared with its row limit, and its source takes
    the scratch address from hipGetSymbolAddress and calls no allocator."""
    src = open(HEADER).read()
    assert "zema_mlp_grad_noalloc" in src and "ZEMA_MLP_NOALLOC_MAX_ROWS" in src
    k = open(os.path.join(ROOT, "paper_2311_05945_amd", "csrc", "k_mlp.hip")).read()
    body = k[k.index("double mlp_grad_noalloc"):]
    body = body[:body.index("\n}\n")]
    assert "hipMalloc" not in body and "reserve" not in body and "resize" not in body
    assert "hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))" in k
