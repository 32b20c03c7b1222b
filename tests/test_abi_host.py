"""C ABI contract checks that need no GPU: the library loads, exports every
entry point include/smx.h declares, and rejects invalid host input before it
touches the device."""
import ctypes as C
import os
import sys
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smx.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smx_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def smx():
    import paper_2606_27086_amd as smx

    if not os.path.exists(smx.LIB_PATH):
        pytest.fail("libsmx.so is not built: run __graft_entry__.build()")
    smx.lib()
    return smx


def test_exports_every_declared_symbol(smx):
    declared = _declared()
    assert len(declared) >= 15
    raw = C.CDLL(smx.LIB_PATH)
    for name in declared:
        assert hasattr(raw, name), name
    assert sorted(smx.EXPORTS) == declared


def test_version(smx):
    assert smx.version() == (0, 1)


def test_footprint_without_device(smx):
    b1 = smx.footprint(1000, 500, 20000, "f32")
    b2 = smx.footprint(1000, 500, 20000, "bf16", keep_f32=False)
    b3 = smx.footprint(1000, 500, 20000, "bf16", keep_f32=True)
    assert b2 < b1 < b3
    with pytest.raises(smx.SmxError) as e:
        smx.footprint(0, 5, 5)
    assert e.value.code == smx.EINVAL


def _csr_call(smx, m, n, rp, ci, val, storage=0):
    rp = np.ascontiguousarray(rp, np.int32)
    ci = np.ascontiguousarray(ci, np.int32)
    val = np.ascontiguousarray(val, np.float32)
    csr = smx.Csr(m, n, ci.size, rp.ctypes.data, ci.ctypes.data if ci.size else None,
                  val.ctypes.data if val.size else None, 0)
    h = C.c_void_p()
    rc = smx.lib().smx_operator_create(C.byref(csr), storage, 1, None, C.byref(h))
    return rc, smx.lib().smx_last_error().decode(), h


@pytest.mark.parametrize(
    "case",
    [
        ("m0", 0, 3, [0], [], []),
        ("no_nonzeros", 2, 3, [0, 0, 0], [], []),
        ("nnz_mismatch", 2, 3, [0, 1, 3], [0, 1], [1.0, 2.0]),
        ("decreasing", 2, 3, [0, 2, 1], [0, 1], [1.0, 2.0]),
        ("col_range", 2, 3, [0, 1, 2], [0, 3], [1.0, 2.0]),
        ("col_negative", 2, 3, [0, 1, 2], [0, -1], [1.0, 2.0]),
        ("nan_value", 2, 3, [0, 1, 2], [0, 1], [1.0, np.nan]),
        ("rowptr0", 2, 3, [1, 1, 2], [0, 1], [1.0, 2.0]),
    ],
)
def test_invalid_csr_rejected_on_host(smx, case):
    name, m, n, rp, ci, val = case
    rc, msg, h = _csr_call(smx, m, n, rp, ci, val)
    assert rc == smx.EINVAL, (name, rc, msg)
    assert msg
    assert not h.value


def test_bad_storage_rejected(smx):
    rc, msg, _ = _csr_call(smx, 2, 2, [0, 1, 2], [0, 1], [1.0, 2.0], storage=7)
    assert rc == smx.EINVAL and "storage" in msg


def test_null_arguments(smx):
    L = smx.lib()
    assert L.smx_operator_create(None, 0, 1, None, None) == smx.EINVAL
    assert L.smx_run(None, 3, 0) == smx.EINVAL
    assert L.smx_query(None, None, None) == smx.EINVAL
    assert L.smx_problem_destroy(None) == smx.OK
    assert L.smx_operator_destroy(None) == smx.OK
    assert L.smx_version(None, None) == smx.EINVAL


def test_binding_has_no_oracle_dependency():
    """The product binding never imports the oracle package."""
    src = open(os.path.join(ROOT, "paper_2606_27086_amd", "__init__.py")).read()
    assert "oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_2606_27086_amd", "csrc")):
        text = open(os.path.join(ROOT, "paper_2606_27086_amd", "csrc", f)).read()
        assert "oracle" not in text and "liborc" not in text and "orc_" not in text


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library the binding raises on first use: there is no
    other path to the kernels."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_2606_27086_amd as smx\n"
        "smx.LIB_PATH = %r\n"
        "try:\n"
        "    smx.lib()\n"
        "except ImportError as e:\n"
        "    print('raised', e)\n"
        "else:\n"
        "    sys.exit(3)\n"
    ) % (ROOT, str(tmp_path / "absent" / "libsmx.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "raised" in r.stdout and "libsmx.so not found" in r.stdout


def test_struct_layouts_match_header(smx, tmp_path):
    """Every ctypes structure of the binding has the size and field offsets the
    C compiler gives the header's structure."""
    structs = {"smx_csr": smx.Csr, "smx_dvc": smx.DvcC, "smx_problem_desc": smx.ProblemDesc,
               "smx_slice_state": smx.SliceStateC}
    header_names = {  # binding field -> header field, where they differ
        "smx_problem_desc": {"lam": "lambda"},
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            hf = header_names.get(cname, {}).get(f, f)
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {hf}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess

    subprocess.check_call(["gcc", "-std=c11", "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        cname, f, v = line.split()
        py = structs[cname]
        want = C.sizeof(py) if f == "size" else getattr(py, f).offset
        assert int(v) == want, (cname, f, int(v), want)
        seen += 1
    assert seen == sum(len(p._fields_) + 1 for p in structs.values())


@pytest.mark.parametrize("shape", [(0, 6), (2, 2), (3, 3), (-1, -6), (6, 0)])
def test_image_shape_rejected_on_host(smx, shape):
    """smx_operator_create_image checks that the image covers exactly n
    unknowns before it touches the device."""
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 5, 1, 2], np.int32)
    val = np.ones(4, np.float32)
    csr = smx.Csr(2, 6, 4, rp.ctypes.data, ci.ctypes.data, val.ctypes.data, 0)
    h = C.c_void_p()
    rc = smx.lib().smx_operator_create_image(C.byref(csr), 0, 1, shape[0], shape[1], None, C.byref(h))
    assert rc == smx.EINVAL and "image" in smx.lib().smx_last_error().decode()
    assert not h.value


def test_problem_footprint_without_device(smx):
    """The problem's share of smx_footprint grows with the slots and with the
    buffers a basic algorithm, the history and the stopping rules add; invalid
    descriptor fields are rejected."""
    ob, p1 = smx.problem_footprint(5000, 3000, 60000, "f32", B=1)
    _, p8 = smx.problem_footprint(5000, 3000, 60000, "f32", B=8)
    _, pe = smx.problem_footprint(5000, 3000, 60000, "f32", B=1, basic=4)
    _, ph = smx.problem_footprint(5000, 3000, 60000, "f32", B=1, history_cap=100)
    _, pv = smx.problem_footprint(5000, 3000, 60000, "f32", B=1, stop=dict(var=1e-3))
    assert ob == smx.footprint(5000, 3000, 60000, "f32")
    assert p8 > 8 * 4 * (2 * 5000 + 2 * 3000) and p1 < p8
    assert pe - p1 >= 8 * 3000 + 4 * 3000 + 4 * 5000 and ph - p1 == 100 * (3 * 8 + 2 * 4)
    assert pv - p1 >= 4 * 3000
    for bad in (dict(B=3), dict(basic=9), dict(obj=2, tv_rows=7, tv_cols=7), dict(history_cap=-1),
                dict(dvc=[dict(row_begin=0, row_end=6000, sense=0, fraction=0.5, dose=1.0)])):
        with pytest.raises(smx.SmxError) as e:
            smx.problem_footprint(5000, 3000, 60000, "f32", **bad)
        assert e.value.code == smx.EINVAL, bad
