"""The C-ABI library loads, exports every declared symbol and rejects bad arguments
before touching a device (CPU only)."""
import ctypes as C
import os
import re

import pytest

from paper_2212_10733_amd import hcz

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "hcz.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hcz_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(hcz.LIB, n), n
    assert sorted(hcz.EXPORTS) == names


def test_version_and_last_error():
    assert hcz.LIB.hcz_version().decode().startswith("hcz")
    assert isinstance(hcz.LIB.hcz_last_error(), bytes)


def test_struct_layouts_match_header(tmp_path):
    # compile the header with the host C compiler and compare sizes and offsets with ctypes
    import subprocess
    src = tmp_path / "layout.c"
    fields = {"hcz_params": hcz.Params, "hcz_grid": hcz.Grid, "hcz_stats": hcz.Stats,
              "hcz_compressed": hcz.CompressedC, "hcz_codebook": hcz.Codebook, "hcz_model_desc": hcz.ModelDesc}
    cname = {"lambda_": "lambda"}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for st, cls in fields.items():
        lines.append(f'  printf("{st} %zu\\n", sizeof({st}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{st}.{f} %zu\\n", offsetof({st}, {cname.get(f, f)}));')
    lines.append("  return 0; }")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                          check=True).stdout.split("\n") if l)
    for st, cls in fields.items():
        assert int(out[st]) == C.sizeof(cls), st
        for f, _ in cls._fields_:
            assert int(out[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)


def bad_grid(**kw):
    g = dict(n_par=39, n_perp=39, vpar_lo=-4.0, vpar_hi=4.0, vperp_lo=0.0, vperp_hi=4.0, mass=1.0)
    g.update(kw)
    return hcz.Grid(g["n_par"], g["n_perp"], g["vpar_lo"], g["vpar_hi"], g["vperp_lo"], g["vperp_hi"], g["mass"], None)


@pytest.mark.parametrize("kw", [dict(n_par=2), dict(n_perp=200), dict(n_par=100, n_perp=100),
                                dict(vpar_hi=-5.0), dict(mass=0.0), dict(vperp_hi=float("nan"))])
def test_plan_rejects_bad_grids(kw):
    ctx = C.c_void_p(1)   # never dereferenced: validation happens first
    out = C.c_void_p()
    g = bad_grid(**kw)
    assert hcz.LIB.hcz_plan_create(ctx, C.byref(g), C.byref(out)) == -1
    assert out.value is None
    assert hcz.LIB.hcz_last_error()


def test_null_arguments_are_rejected():
    L = hcz.LIB
    assert L.hcz_create(0, None) == -1
    assert L.hcz_plan_create(None, None, None) == -1
    assert L.hcz_qoi(None, None, 0, 1, 1521, 39, None, None, None, None) == -1
    assert L.hcz_encode(None, None, 0, 1, 1521, 39, None, None) == -1
    assert L.hcz_residual(None, None, None, 0, 1, 1521, 39, None, None, None, None, 0, None) == -1
    assert L.hcz_compress(None, None, None, None, None, 0, 1, 1521, 39, None, None, 0, None) == -1
    assert L.hcz_decompress(None, None, None, None, 0, 1, None, 1, None, 0, None) == -1
    assert L.hcz_stats_read(None, None, None) == -1
    n = C.c_size_t()
    assert L.hcz_codebook_fit_workspace(0, 16, 1, C.byref(n)) == -1
    assert L.hcz_codebook_fit_workspace(100, 16, 1, C.byref(n)) == 0 and n.value > 100 * 16 * 4
    cb = hcz.Codebook(9, 1)
    assert L.hcz_quantize(C.c_void_p(1), 1, 16, C.byref(cb), C.c_void_p(1), None) == -1   # bits > 8
