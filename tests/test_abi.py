"""The C interface without a GPU: the library builds, loads, and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wc_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["wc_create_gauge", "wc_create_clover", "wc_apply_D", "wc_sap_block_mr", "wc_fgcr_solve",
                 "wc_fgcr_solve_batch", "wc_force", "wc_link_grad", "wc_destroy", "wc_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1109_4279_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwc.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    # the Python binding declares exactly the header's entry points
    assert sorted(_lib.exported_symbols()) == _declared()
    lib2 = _lib.load()
    assert lib2.wc_version() == 201


def _param_counts():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for name, params in re.findall(r"\b(wc_[A-Za-z0-9_]+)\s*\(([^)]*)\)\s*;", text):
        params = params.strip()
        out[name] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_argument_counts_match_header():
    from paper_1109_4279_amd import _lib
    counts = _param_counts()
    assert set(counts) == set(_declared())
    for name, (_, args) in _lib._SIGS.items():
        assert len(args) == counts[name], name


def _struct_fields(name):
    """Field names of the C struct `name` in include/wc.h, in declaration order."""
    src = open(os.path.join(ROOT, "include", "wc.h")).read()
    end = re.search(r"\}\s*" + name + ";", src).start()
    body = src[src.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    decls = [re.sub(r"\[[^\]]*\]\s*$", "", d.strip()) for d in body.split(";") if d.strip()]
    return [re.findall(r"(\w+)\s*$", d)[0] for d in decls]


def test_binding_structs_match_header():
    from paper_1109_4279_amd import _lib
    assert [f for f, _ in _lib.SolverParams._fields_] == _struct_fields("wc_solver_params")
    assert [f for f, _ in _lib.SolverStats._fields_] == _struct_fields("wc_solver_stats")
    src = open(HEADER).read()
    assert int(re.search(r"#define WC_HIST_MAX (\d+)", src).group(1)) == _lib.HIST_MAX
    for name, value in _lib.OPTIONS.items():
        assert re.search(r"WC_OPT_%s = %d\b" % (name.upper(), value), src), name


def test_struct_sizes_match_a_c_compiler(tmp_path):
    """sizeof and field offsets of the two parameter structs as gcc lays them out equal the
    ctypes layout the binding uses."""
    import shutil
    import subprocess
    from paper_1109_4279_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    lines = []
    for cname, py in (("wc_solver_params", _lib.SolverParams), ("wc_solver_stats", _lib.SolverStats)):
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"wc.h\"\nint main(void) {\n"
                   + "\n".join(lines) + "\n  return 0;\n}\n")
    exe = tmp_path / "layout"
    cc = subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                        capture_output=True, text=True, timeout=120)
    assert cc.returncode == 0, cc.stderr
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                               timeout=60).stdout.splitlines())
    for cname, py in (("wc_solver_params", _lib.SolverParams), ("wc_solver_stats", _lib.SolverStats)):
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_default_params_and_error_text():
    from paper_1109_4279_amd import _lib, default_params
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwc.so not built")
    p = default_params()
    assert (p.nkv, p.ncy, p.nmr, p.sap_prec, p.maxit, p.eo, p.dagger, p.stag, p.timing) == \
        (16, 5, 4, 1, 10000, 0, 0, 3, 0)
    assert abs(p.tol - 1e-10) < 1e-25
    assert (p.basis_prec, p.drop) == (0, 0.0)  # FP64 Krylov basis, no per-cycle drop
    q = default_params(basis_prec="f32", drop=1e-6)
    assert (q.basis_prec, q.drop) == (1, 1e-6)
    lib = _lib.load()
    # argument errors are reported without touching a device
    ctx = ctypes.c_void_p()
    dims = (ctypes.c_int * 4)(4, 4, 4, 4)
    blk = (ctypes.c_int * 4)(2, 2, 2, 2)
    assert lib.wc_create_gauge(ctypes.byref(ctx), dims, blk, None, 1, None) == -1
    assert b"null" in lib.wc_last_error()
    assert lib.wc_create_gauge(ctypes.byref(ctx), dims, blk, ctypes.c_void_p(16), 3, None) == -1
    assert lib.wc_apply_D(None, None, None, 1, 0, 0, 0, None) == -1


def test_solver_params_from_keywords():
    """Keywords replace fields of the defaults or of a given parameter block (which is
    copied, never changed); a name that is not a field is an error, not ignored."""
    from paper_1109_4279_amd import _lib, _params, default_params
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwc.so not built")
    p = default_params(nkv=8, sap_prec="f16")
    assert (p.nkv, p.sap_prec) == (8, _lib.PREC["f16"])
    q = _params(p, {"tol": 1e-8, "eo": 1})
    assert (q.tol, q.eo, q.nkv) == (1e-8, 1, 8)
    assert (p.tol, p.eo) == (1e-10, 0)
    assert _params(None, {"nmr": 2}).nmr == 2
    with pytest.raises(TypeError, match="tolerance"):
        default_params(tolerance=1e-8)
    with pytest.raises(TypeError, match="nvk"):
        _params(p, {"nvk": 3})


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1109_4279_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", src, flags=re.M), f
                assert "oracle/" not in src, f


def test_header_is_c99_and_links(tmp_path):
    """A C99 client (-Wall -Wextra -pedantic -Werror) that includes only wc.h, takes the
    address of every declared entry point and links against libwc.so: the header is plain C
    and the library resolves every symbol at link time.  Run, it checks the defaults and two
    argument errors, which touch no device."""
    import shutil
    import subprocess
    from paper_1109_4279_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libwc.so not built")
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    refs = "\n".join(f"  (void (*)(void)){n}," for n in _declared())
    src = tmp_path / "client.c"
    src.write_text(f"""#include <stdio.h>
#include <string.h>
#include "wc.h"
static void (*const entry_points[])(void) = {{
{refs}
}};
int main(void) {{
  wc_ctx* ctx = NULL;
  const int dims[4] = {{4, 4, 4, 4}}, block[4] = {{2, 2, 2, 2}};
  wc_solver_params p;
  size_t i;
  for (i = 0; i < sizeof entry_points / sizeof entry_points[0]; ++i)
    if (!entry_points[i]) return 1;
  wc_default_params(&p);
  if (p.nkv != 16 || p.eo != 0 || p.dagger != 0) return 2;
  if (wc_create_gauge(&ctx, dims, block, NULL, 1, NULL) != WC_ERR_ARG || strlen(wc_last_error()) == 0) return 3;
  if (wc_fgcr_solve(NULL, NULL, NULL, 1, &p, NULL, NULL) != WC_ERR_ARG) return 4;
  printf("%d\\n", wc_version());
  return 0;
}}
""")
    lib_dir = os.path.dirname(_lib.LIB_PATH)
    exe = tmp_path / "client"
    cc = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                         str(src), "-L", lib_dir, "-lwc", f"-Wl,-rpath,{lib_dir}", "-o", str(exe)],
                        capture_output=True, text=True, timeout=120)
    assert cc.returncode == 0, cc.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert run.returncode == 0, (run.returncode, run.stderr)
    assert run.stdout.strip() == "201"
