"""The C-ABI library loads on the host and exports every entry point that
include/afqmc.h declares (no compute calls: no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afqmc.h")
LIB = os.path.join(ROOT, "paper_1703_01545_amd", "libafqmc.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(afqmc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ("afqmc_load_hamiltonian", "afqmc_init_walkers", "afqmc_step",
                     "afqmc_local_energy", "afqmc_orthonormalize", "afqmc_pair_step"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libafqmc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libafqmc.so not built")
def test_binding_lists_every_declared_symbol():
    from paper_1703_01545_amd import afqmc
    assert sorted(afqmc.EXPORTS) == declared()


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_1703_01545_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.sub(r"(#|//).*", "", text), f


@pytest.mark.skipif(not os.path.exists(LIB), reason="libafqmc.so not built")
def test_tune_cache_load_rejects_files_that_are_not_caches(tmp_path):
    """The format is checked before anything asks for a device."""
    from paper_1703_01545_amd import afqmc
    bad = tmp_path / "notes.txt"
    bad.write_text("not a tune cache\n")
    for path in (str(tmp_path / "missing"), str(bad)):
        with pytest.raises(afqmc.AfqmcError) as e:
            afqmc.tune_cache_load(path)
        assert e.value.status == afqmc.E_INVALID
