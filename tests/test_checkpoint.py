"""Predictor checkpoints (host only): the parameters travel with a layout
record and their provenance, and a file for another layout, a wrong size or
altered parameters is refused."""

import json

import numpy as np
import pytest

from paper_2108_11560_amd import mlp as M


def params(seed=0):
    return M.glorot_params(seed, margins=(0.02, 0.04))


PROV = {"train": {"steps": 100, "seed": 7, "batch": 512}, "labels": {"sha256_t0_t1": "ab" * 32},
        "margins": {"t1": 0.02, "t0": 0.04}}


def test_roundtrip(tmp_path):
    path = str(tmp_path / "net.bin")  # any suffix: the exact path is written
    p = params()
    M.write_checkpoint(path, p, PROV)
    q, prov = M.read_checkpoint(path)
    assert q.dtype == np.float32 and np.array_equal(q, p)
    assert prov == PROV


def test_refuses_a_plain_parameter_array(tmp_path):
    path = str(tmp_path / "old.npy")
    np.save(path, params())
    with pytest.raises(ValueError, match="no layout record"):
        M.read_checkpoint(path)


def rewrite(path, **changes):
    with np.load(path, allow_pickle=False) as f:
        arr, meta = np.array(f["params"]), json.loads(str(f["meta"]))
    arr = changes.pop("params", arr)
    meta.update(changes)
    with open(path, "wb") as fh:
        np.savez(fh, params=arr, meta=np.array(json.dumps(meta)))


@pytest.mark.parametrize("change, match", [
    ({"layout": "2-64-64-2 tanh"}, "layout"),
    ({"version": 0}, "layout or format version"),
    ({"nparams": 4482}, "parameters"),
])
def test_refuses_other_layouts_and_sizes(tmp_path, change, match):
    path = str(tmp_path / "net.npz")
    M.write_checkpoint(path, params(), PROV)
    rewrite(path, **change)
    with pytest.raises(ValueError, match=match):
        M.read_checkpoint(path)


def test_refuses_altered_parameters(tmp_path):
    path = str(tmp_path / "net.npz")
    p = params()
    M.write_checkpoint(path, p, PROV)
    q = p.copy()
    q[17] += 1e-3
    rewrite(path, params=q)
    with pytest.raises(ValueError, match="hash"):
        M.read_checkpoint(path)


def test_wrong_size_is_refused_on_write(tmp_path):
    with pytest.raises(ValueError):
        M.write_checkpoint(str(tmp_path / "x.npz"), np.zeros(10, np.float32), None)
