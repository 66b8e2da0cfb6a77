"""The model file (dpk_model_load / dpk_model_save): a versioned JSON header and the FP64 blob.

Host-only (no GPU): a round trip keeps the description and every parameter bit for bit, and the
table's stride and range of a compressed model (its table is rebuilt at load); writing a loaded
model gives the same bytes; malformed files are refused with DPK_E_INVALID_ARG. That a loaded model
evaluates bit for bit like the model it was saved from is a GPU test (test_gpu_model_file.py).
"""
import json
import os
import struct

import numpy as np
import pytest

from paper_2304_09409_amd import dpk, synth


def _header(path):
    with open(path, "rb") as f:
        raw = f.read()
    assert raw[:8] == b"DPKMODEL"
    (hl,) = struct.unpack("<Q", raw[8:16])
    return raw, json.loads(raw[16:16 + hl].decode()), 16 + hl + (8 - (16 + hl) % 8) % 8


@pytest.mark.parametrize("spec,params,table", [
    (synth.WATER_MODEL, synth.water_params, None),
    (synth.FCC_MODEL, synth.fcc_params, (0.01, 0.5)),
    (dict(synth.SERVE_MODEL, type_one_side=True), None, None),
    (synth.WATER_R_MODEL, synth.water_r_params, (0.005, 2.0)),
    (synth.WATER_E3_MODEL, synth.water_e3_params, (0.01, 8.0)),
])
def test_round_trip(tmp_path, spec, params, table):
    p = params() if params else synth.make_params(spec, 9, timestep_sigma=0.1)
    m = dpk.Model(spec, p)
    if table:
        m.tabulate(*table)
    path = str(tmp_path / "model.dpk")
    m.save(path)
    raw, head, off = _header(path)
    assert head["format"] == "dpk-se_e2_a" and head["version"] == 1 and head["nparams"] == p.size
    # the blob is the parameters as little-endian binary64, bit for bit
    np.testing.assert_array_equal(np.frombuffer(raw[off:], dtype="<f8"), p)
    m2 = dpk.Model.load(path)
    d, p2, stride, xmax = m2.describe()
    assert d == dict(spec, type_one_side=bool(spec["type_one_side"]))
    assert p2.tobytes() == p.tobytes()
    assert (stride, xmax) == (table if table else (0.0, 0.0))
    path2 = str(tmp_path / "again.dpk")
    m2.save(path2)
    assert open(path, "rb").read() == open(path2, "rb").read()


def test_malformed_files_are_refused(tmp_path):
    m = dpk.Model(synth.WATER_MODEL, synth.water_params())
    good = str(tmp_path / "good.dpk")
    m.save(good)
    raw, head, off = _header(good)

    def write(name, data):
        path = str(tmp_path / name)
        with open(path, "wb") as f:
            f.write(data)
        return path

    def with_header(h):
        js = json.dumps(h).encode()
        pad = (8 - (16 + len(js)) % 8) % 8
        return b"DPKMODEL" + struct.pack("<Q", len(js)) + js + b"\0" * pad + raw[off:]

    cases = {
        "magic": b"NOTMODEL" + raw[8:],
        "truncated_blob": raw[:-8],
        "truncated_header": raw[:20],
        "version": with_header(dict(head, version=2)),
        "format": with_header(dict(head, format="other")),
        "nparams": with_header(dict(head, nparams=head["nparams"] + 1)),
        "missing_key": with_header({k: v for k, v in head.items() if k != "rcut"}),
        "sel_type": with_header(dict(head, sel=[46.5, 92])),
        "not_json": b"DPKMODEL" + struct.pack("<Q", 5) + b"{abc}" + b"\0" * 3 + raw[off:],
    }
    for name, data in cases.items():
        with pytest.raises(dpk.DpkError) as e:
            dpk.Model.load(write(name, data))
        assert e.value.code == dpk.DPK_E_INVALID_ARG, name
    with pytest.raises(dpk.DpkError):
        dpk.Model.load(str(tmp_path / "missing.dpk"))
    # a header that names a compressed model rebuilds its table
    t = dpk.Model.load(write("tab", with_header(dict(head, compression={"stride": 0.02, "x_max": 2.0}))))
    assert t.describe()[2:] == (0.02, 2.0)
