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


def _header_enum_values():
    text = HEADER.read_text()
    vals = {m.group(1): 1 << int(m.group(2)) for m in re.finditer(r"\b(QED_[A-Z0-9_]+)\s*=\s*1u\s*<<\s*(\d+)", text)}
    for m in re.finditer(r"\b(QED_FIELD_[A-Z0-9_]+)\s*=\s*(\d+)", text):
        vals[m.group(1)] = int(m.group(2))
    return vals


def test_flag_values_agree_across_header_binding_and_oracle():
    """The physics switches and field models have one meaning everywhere: the header's values,
    the binding's constants and the oracle's (whose flag words the tests pass straight through)."""
    import oracle
    import paper_2511_08929_amd as q
    hv = _header_enum_values()
    assert len(hv) >= 19
    for name, v in hv.items():
        assert getattr(q, name) == v, name
    pairs = {"QED_PUSH": "F_PUSH", "QED_TBMT": "F_TBMT", "QED_EMIT": "F_EMIT", "QED_RECOIL": "F_RECOIL",
             "QED_SPIN": "F_SPIN", "QED_NOEMIT": "F_NOEMIT", "QED_PHOTON_POL": "F_PHOTON_POL", "QED_MEAN": "F_MEAN",
             "QED_PAIR": "F_PAIR", "QED_NOPAIR": "F_NOPAIR", "QED_PAIR_SPIN": "F_PAIR_SPIN",
             "QED_OPTICAL_DEPTH": "F_TAU", "QED_REJECTION": "F_REJECT", "QED_G_CHI": "F_GCHI",
             "QED_SUBCYCLE": "F_SUB", "QED_FIELD_UNIFORM": "FIELD_UNIFORM", "QED_FIELD_PLANE_LP": "FIELD_PLANE_LP",
             "QED_FIELD_GRID2D": "FIELD_GRID2D", "QED_FIELD_ROTATING_E": "FIELD_ROTATING_E"}
    for h, o in pairs.items():
        assert hv[h] == getattr(oracle, o), (h, o)
    assert q.QED_ALL == oracle.F_ALL
