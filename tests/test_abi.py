"""CPU checks of the C ABI library: it loads and exports every entry point include/qedspin.h declares.
No compute call is made (there may be no GPU)."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "qedspin.h"


def declared_symbols():
    text = HEADER.read_text()
    return sorted(set(re.findall(r"^\s*(?:qed_status|size_t|int64_t|const char \*)\s*(qed_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for n in ("qed_init_tables", "qed_push_spin", "qed_emit", "qed_pair", "qed_compact"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2511_08929_amd as q
    if not q.LIB_PATH.exists():
        pytest.fail("libqedspin.so is not built (run paper_2511_08929_amd/build.py)")
    lib = ctypes.CDLL(str(q.LIB_PATH))
    for n in declared_symbols():
        assert hasattr(lib, n), n
    assert set(declared_symbols()) == set(q.ABI_SYMBOLS)


def test_binding_has_no_cpu_fallback(tmp_path, monkeypatch):
    import paper_2511_08929_amd as q
    monkeypatch.setattr(q, "LIB_PATH", tmp_path / "missing.so")
    monkeypatch.setattr(q, "_lib", None)
    with pytest.raises(q.QedError):
        q.lib()
