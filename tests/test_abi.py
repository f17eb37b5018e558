"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every function
include/pond.h declares, and the binding's symbol list matches the header."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pond.h")
LIB = os.path.join(ROOT, "paper_2203_05477_amd", "libpond.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pond_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib_symbols():
    if not os.path.exists(LIB):
        from paper_2203_05477_amd import build

        build.build()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    return {line.split()[-1] for line in out.splitlines() if line.strip()}


def test_header_declares_the_entry_points():
    names = declared()
    for core in ("pond_init", "pond_step", "pond_moments", "pond_free", "pond_strerror"):
        assert core in names
    assert len(names) >= 30


def test_library_exports_every_declared_symbol(lib_symbols):
    missing = [n for n in declared() if n not in lib_symbols]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    from paper_2203_05477_amd import pond

    assert sorted(pond.exported_symbols()) == declared()


def test_library_loads_and_reports_abi_version():
    from paper_2203_05477_amd import pond

    lib = pond.load()
    assert lib.pond_abi_version() == 5
    assert lib.pond_strerror(1) == b"invalid argument"
    assert lib.pond_mlp_nparams() == 8515


def test_stats_struct_layout_matches_the_header(tmp_path):
    """The binding's pond_stats and pond_config layouts equal the C compiler's (sizes and
    field offsets), so the summary fields land where the library writes them."""
    import ctypes

    from paper_2203_05477_amd import pond

    fields = {"pond_stats": pond.Stats, "pond_config": pond.Config}
    src = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){"]
    for cname, cls in fields.items():
        src.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for name, _ in cls._fields_:
            src.append(f'printf("{cname} {name} %zu\\n", offsetof({cname}, {name}));')
    src.append("return 0;}")
    (tmp_path / "layout.c").write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(tmp_path / "layout.c")], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in fields.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls)
        for name, _ in cls._fields_:
            assert got[(cname, name)] == getattr(cls, name).offset, (cname, name)
