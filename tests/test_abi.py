"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent


def declared_functions():
    text = (ROOT / "include" / "eloc.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(eloc_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("eloc_create", "eloc_set_hamiltonian", "eloc_set_samples", "eloc_local_energy",
              "eloc_find_pairs", "eloc_pair_elements", "eloc_local_energy_adjoint"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib_path = ROOT / "paper_2408_07625_amd" / "libeloc.so"
    if not lib_path.exists():
        pytest.fail("libeloc.so is not built (python -m paper_2408_07625_amd.build)")
    import torch  # noqa: F401  (the HIP runtime the library binds to)
    lib = ctypes.CDLL(str(lib_path))
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2408_07625_amd as pe
    with pytest.raises(pe.ElocError) as ex:
        pe.Engine(0)
    assert ex.value.status == "EINVAL"


def test_null_arguments_rejected():
    import paper_2408_07625_amd as pe
    lib = pe.library()
    assert lib.eloc_create(None, 0, None) == -1
    assert lib.eloc_set_hamiltonian(None, 4, 1, None, None, None) == -1
    assert lib.eloc_last_error(None) == b"null context"
