"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/rabitq.h declares, and validates arguments and files."""
import os
import re
import struct

import numpy as np
import pytest

from paper_2405_12497_amd import rabitq as R

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "rabitq.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:rbq_status|const char\*)\s+(rbq_\w+)\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = R.lib()
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing
    assert sorted(R.exported_symbols()) == names


def test_params_default_and_validation():
    p = R.rbq_params_default(128, 4096)
    assert (p.dim, p.code_bits, p.nlist, p.bq) == (128, 0, 4096, 4)
    assert abs(p.eps0 - 1.9) < 1e-7
    h = R.rbq_index_create(p)
    info = R.rbq_index_info_get(h)
    assert info["code_bits"] == 128 and info["n"] == 0
    R.rbq_index_destroy(h)
    p2 = R.rbq_params_default(100, 1)
    h2 = R.rbq_index_create(p2)
    assert R.rbq_index_info_get(h2)["code_bits"] == 128     # padded to a multiple of 64
    R.rbq_index_destroy(h2)


@pytest.mark.parametrize("field,value,status", [
    ("dim", 0, R.RBQ_EINVAL), ("dim", 5000, R.RBQ_EINVAL), ("code_bits", 100, R.RBQ_EINVAL),
    ("code_bits", 64, R.RBQ_EINVAL), ("nlist", 0, R.RBQ_EINVAL), ("bq", 0, R.RBQ_EINVAL), ("bq", 9, R.RBQ_EINVAL),
    ("eps0", -1.0, R.RBQ_EINVAL), ("rot_precision", 7, R.RBQ_EINVAL)])
def test_create_rejects_bad_params(field, value, status):
    p = R.rbq_params_default(128, 16)
    setattr(p, field, value)
    with pytest.raises(R.RbqError) as e:
        R.rbq_index_create(p)
    assert e.value.status == status
    assert R.rbq_last_error()


def test_calls_on_unbuilt_index_fail_with_estate():
    h = R.rbq_index_create(R.rbq_params_default(64, 4))
    o = R.RbqSearchOpts(10, 1, 0, 0, None, 0, 0, 0)
    st = R.lib().rbq_search(h, None, 1, o, None, None, None, None)
    assert st == R.RBQ_ESTATE
    assert R.lib().rbq_index_save(h, b"/tmp/never.rbq") == R.RBQ_ESTATE
    assert R.lib().rbq_index_list_sizes(h, np.zeros(4, np.int64).ctypes.data) == R.RBQ_ESTATE
    R.rbq_index_destroy(h)
    assert R.lib().rbq_index_destroy(None) == R.RBQ_EINVAL


def test_load_rejects_missing_bad_and_truncated_files(tmp_path):
    with pytest.raises(R.RbqError) as e:
        R.rbq_index_load(str(tmp_path / "none.rbq"))
    assert e.value.status == R.RBQ_EINVAL
    bad = tmp_path / "bad.rbq"
    bad.write_bytes(b"NOTANIDX" + b"\0" * 64)
    with pytest.raises(R.RbqError) as e:
        R.rbq_index_load(str(bad))
    assert e.value.status == R.RBQ_EFORMAT
    # valid header, payload cut short
    hdr = b"RBQIDX01" + struct.pack("<IiiiiifIQq", 1, 64, 64, 2, 4, 0, 1.9, 0, 0, 10)
    trunc = tmp_path / "trunc.rbq"
    trunc.write_bytes(hdr + b"\0" * 100)
    with pytest.raises(R.RbqError) as e:
        R.rbq_index_load(str(trunc))
    assert e.value.status == R.RBQ_EFORMAT
