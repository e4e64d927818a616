"""The C-ABI library loads and exports every entry point include/hopfpd.h
declares; host-side argument handling that needs no GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1712_08226_amd import hopfpd as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "hopfpd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hopf_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = H.load()
    decl = declared_symbols()
    assert len(decl) >= 16
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(H.EXPORTS)


def test_strerror_and_defaults_without_gpu():
    lib = H.load()
    assert lib.hopf_strerror(0) == b"ok"
    assert lib.hopf_strerror(1) == b"invalid argument"
    o = H.default_opts()
    assert o.gap_tol == 1e-6 and o.t_rel_tol == 0.5e-4 and o.check_every > 0


def test_null_context_is_rejected():
    lib = H.load()
    assert lib.hopf_set_opts(None, None) == 1
    assert lib.hopf_last_error(None) == b"null context"
    lib.hopf_destroy(None)                      # no-op


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="host without a GPU only")
def test_create_without_device_reports_device_error():
    lib = H.load()
    h = C.c_void_p()
    assert lib.hopf_create(0, C.byref(h)) == 3
    assert not h.value


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding have the sizes and field offsets
    of the C structures in include/hopfpd.h (compiled here with gcc)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"hopf_opts": H.HopfOpts, "hopf_system": H.HopfSystem, "hopf_timing": H.HopfTiming}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{os.path.join(ROOT, "include", "hopfpd.h")}"',
             "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_set_opts_rejects_unknown_option_names():
    """A misspelt option must not be dropped silently (ctypes structures
    accept any attribute); the check runs before the library is called."""
    class NoCtx:
        pass
    with pytest.raises(TypeError, match="unknown solver option"):
        H.Solver.set_opts(NoCtx(), wide_minn=1)


def test_documented_option_defaults_match_the_library():
    """Every numeric default the header documents in brackets after an option
    is the value hopf_default_opts fills in."""
    txt = open(os.path.join(ROOT, "include", "hopfpd.h")).read()
    block = txt[txt.index("/* Solver options"):txt.index("} hopf_opts;")]
    names = [f[0] for f in H.HopfOpts._fields_]
    o = H.default_opts()
    # option name at the start of a doc line, then the text up to the next option
    starts = [(m.start(), m.group(1)) for m in re.finditer(r"\n \*   ([a-z_0-9]+) ", block) if m.group(1) in names]
    checked = 0
    for (pos, name), nxt in zip(starts, starts[1:] + [(len(block), None)]):
        brackets = re.findall(r"\[([^\]]*)\]\s*(?:\n|\*/|$)", block[pos:nxt[0]])
        if not brackets:
            continue
        vals = [v.strip() for v in brackets[-1].split(",")]
        try:
            nums = [float(v) for v in vals]
        except ValueError:
            continue                      # symbolic default (an enum name)
        if len(nums) == 1:
            assert getattr(o, name) == nums[0], (name, getattr(o, name), nums[0])
            checked += 1
        elif name == "t_abs_frac":      # the pair t_rel_tol, t_abs_frac is documented on its line
            assert (o.t_rel_tol, o.t_abs_frac) == tuple(nums), (o.t_rel_tol, o.t_abs_frac, nums)
            checked += 2
    assert checked >= 12, checked
