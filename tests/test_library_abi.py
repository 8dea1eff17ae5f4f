"""Host-side checks of the C-ABI library: it loads and exports every symbol the
header declares; size queries and argument validation work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1605_03228_amd import binding
    if not os.path.exists(binding.library_path()):
        from paper_1605_03228_amd.build import build
        build()
    return binding.load()


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "ihdg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ihdg_\w+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n


def test_sizes(lib):
    from paper_1605_03228_amd import binding as b
    s = b.sizes((256, 256), 4, b.TRANSPORT)
    assert s["n_el"] == 65536 and s["np"] == 25 and s["n_loc"] == 25 and s["n_in"] == 20
    assert s["nq"] == 36 and s["nfq"] == 6 and s["n_face"] == 2 * 257 * 256
    s = b.sizes((64, 64, 64), 3, b.TRANSPORT)
    assert s["n_loc"] == 64 and s["n_in"] == 96 and s["n_face"] == 3 * 65 * 64 * 64
    s = b.sizes((128, 128), 3, b.SHALLOW_WATER)
    assert s["n_loc"] == 48 and s["n_in"] == 16 and s["m_f"] == 3
    s = b.sizes((128, 128), 4, b.CD)
    assert s["n_loc"] == 75 and s["n_in"] == 20


def test_argument_validation(lib):
    from paper_1605_03228_amd import binding as b
    with pytest.raises(b.IhdgError) as e:
        b.sizes((8, 8), 0, b.TRANSPORT)
    assert e.value.status == 2
    with pytest.raises(b.IhdgError) as e:
        b.sizes((8, 8, 8), 3, b.SHALLOW_WATER)
    assert e.value.status == 2
    with pytest.raises(b.IhdgError) as e:
        b.sizes((8, 8), 7, b.CD)
    assert e.value.status == 2
    assert lib.ihdg_sizes(None, 2, 0, None) == 1


def test_footprint_shared_vs_per_element(lib):
    from paper_1605_03228_amd import binding as b
    shared, _ = b.footprint((64, 64), 4, b.TRANSPORT, {"beta_const": (1.0, 0.5)})
    per, _ = b.footprint((64, 64), 4, b.TRANSPORT, {"beta_const": (1.0, 0.5)}, force_per_element=True)
    assert per > shared + 4096 * 25 * 20 * 8 * 0.9
    mixed, _ = b.footprint((64, 64), 4, b.TRANSPORT, None, prec=b.MIXED)
    assert mixed > per


def test_mesh_limits(lib):
    """Empty meshes are rejected as invalid arguments; meshes above 2^30
    elements (the limit of the int32 face map times 64-element blocks) as
    unsupported."""
    from paper_1605_03228_amd import binding as b
    for n in [(0, 5), (5, 0), (3, 0, 3)]:
        with pytest.raises(b.IhdgError) as e:
            b.sizes(n, 2, b.TRANSPORT)
        assert e.value.status == 1, n
    with pytest.raises(b.IhdgError) as e:
        b.sizes((1 << 11, 1 << 11, 1 << 9), 1, b.TRANSPORT)  # 2^31 elements
    assert e.value.status == 2
    s = b.sizes((1 << 15, 1 << 15), 1, b.TRANSPORT)           # exactly 2^30 elements
    assert s["n_el"] == 1 << 30
    s = b.sizes((1, 1), 6, b.CD)
    assert s["n_el"] == 1 and s["n_loc"] == 3 * 49 and s["n_in"] == 28


def test_struct_layouts_match_the_header(lib, tmp_path):
    """Every ctypes mirror of a header struct has the size and field offsets a C
    compiler gives it (checked with gcc): a mirror smaller than the struct would
    let the library write past a buffer the binding allocated."""
    import shutil
    import subprocess
    from paper_1605_03228_amd import binding as b
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    mirrors = {"ihdg_mesh": b.Mesh, "ihdg_sizes_t": b.Sizes, "ihdg_coeffs": b.Coeffs,
               "ihdg_options": b.Options, "ihdg_stats": b.Stats, "ihdg_batch_result": b.BatchResult}
    checks = {cname: (cls, [f[0] for f in cls._fields_]) for cname, cls in mirrors.items()}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ihdg.h"', "int main(void) {"]
    for cname, (_, fields) in checks.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, (cls, fields) in checks.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f in fields:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_krylov_option_marshalling(lib):
    from paper_1605_03228_amd import binding as b
    o = b._options(krylov="bicgstab")
    assert o.krylov_method == 1 and o.krylov_restart >= 1
    o = b._options(krylov_restart=40)
    assert o.krylov_method == 0 and o.krylov_restart == 40
    o = b._options()
    assert o.krylov_method == 0 and o.krylov_restart == 0
    with pytest.raises(KeyError):
        b._options(krylov="cg")


def test_serving_routes_elliptic_and_diffusive_requests_to_krylov():
    import workloads as w
    from paper_1605_03228_amd.serving import needs_krylov
    assert needs_krylov(w.cd_elliptic((8, 8), 2, gamma=1.0))
    assert needs_krylov(w.config4b(eps=1e-2, n=8, p=2))
    assert not needs_krylov(w.config4b(eps=1e-4, n=8, p=2))
    assert not needs_krylov(w.config2(n=8, p=2))
