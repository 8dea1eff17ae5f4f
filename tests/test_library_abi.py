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
