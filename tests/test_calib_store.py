"""Host logic of the tagged calibration store and of the closed-loop state
files (no device): keys, staleness, atomic writes, no pickled objects."""
import json
import os

import numpy as np
import pytest

from paper_1607_07624_amd.calib import CalibrationStore, config_hash
from paper_1607_07624_amd.loop import save_state, load_state
from synth.configs import CFG1, CFG2


def test_config_hash_is_stable_and_sensitive():
    v = np.arange(10, dtype=np.int32)
    h = config_hash(CFG1, valid=v, eps_nm=10.0)
    assert h == config_hash(CFG1, eps_nm=10.0, valid=v.copy())            # order of parts, copies
    assert h == config_hash(CFG1.as_dict(), valid=v, eps_nm=10.0)        # record or dict
    assert h != config_hash(CFG2, valid=v, eps_nm=10.0)
    assert h != config_hash(CFG1.with_(n_mod=CFG1.n_mod + 4), valid=v, eps_nm=10.0)
    assert h != config_hash(CFG1, valid=v[:-1], eps_nm=10.0)
    assert h != config_hash(CFG1, valid=v.astype(np.int64), eps_nm=10.0)  # dtype counts
    assert h != config_hash(CFG1, valid=v.reshape(2, 5), eps_nm=10.0)    # shape counts
    assert h != config_hash(CFG1, valid=v, eps_nm=10.000001)
    w = v.copy()
    w[3] += 1
    assert h != config_hash(CFG1, valid=w, eps_nm=10.0)


def test_store_round_trip_and_stale_keys(tmp_path):
    st = CalibrationStore(str(tmp_path / "calib"))
    assert st.tags() == [] and st.load("recmat", "k") is None and st.key_of("recmat") is None
    R = np.random.default_rng(0).normal(size=(6, 14)).astype(np.float32)
    sig = np.linspace(3, 1, 6)
    p = st.save("recmat", "key-1", R=R, sigma=sig, config=np.array(json.dumps({"a": 1})))
    assert os.path.basename(p) == "recmat.npz" and st.tags() == ["recmat"]
    got = st.load("recmat", "key-1")
    assert set(got) == {"R", "sigma", "config"}
    assert np.array_equal(got["R"], R) and got["R"].dtype == np.float32 and np.array_equal(got["sigma"], sig)
    assert st.load("recmat", "key-2") is None                             # stale key never returned
    assert st.key_of("recmat") == "key-1"
    st.save("recmat", "key-2", R=2 * R, sigma=sig)                        # replaced in place
    assert st.load("recmat", "key-1") is None
    assert np.array_equal(st.load("recmat", "key-2")["R"], 2 * R)
    assert not [f for f in os.listdir(st.root) if ".tmp" in f]           # no temporaries left
    with np.load(st.path("recmat"), allow_pickle=False) as z:            # plain arrays only
        assert str(z["_tag"]) == "recmat"


def test_store_rejects_bad_tags_and_reserved_names(tmp_path):
    st = CalibrationStore(str(tmp_path))
    for tag in ("", "../x", "a/b", ".hidden"):
        with pytest.raises(ValueError):
            st.path(tag)
    with pytest.raises(ValueError):
        st.save("ok", "k", _key=np.zeros(1))


def test_store_ignores_other_formats(tmp_path):
    st = CalibrationStore(str(tmp_path))
    os.makedirs(st.root, exist_ok=True)
    np.savez(st.path("recmat"), R=np.zeros(3), _key=np.array("k"))       # no format marker
    assert st.load("recmat", "k") is None


def test_loop_state_file_round_trip(tmp_path):
    cmd = np.random.default_rng(1).normal(size=(2, 60)).astype(np.float32)
    state = {"t": 137, "commands": cmd, "learned": True, "fallback_step": -1,
             "judged": [(0, 0.93), (10, 0.71), (130, float("nan"))]}
    path = str(tmp_path / "loop.npz")
    save_state(path, state, meta={"screen_seed": 5, "offset_px": 39.1})
    got, meta = load_state(path)
    assert got["t"] == 137 and got["learned"] is True and got["fallback_step"] == -1
    assert np.array_equal(got["commands"], cmd) and got["commands"].dtype == np.float32
    assert got["judged"][:2] == [(0, 0.93), (10, 0.71)] and np.isnan(got["judged"][2][1])
    assert meta == {"screen_seed": 5, "offset_px": 39.1}
    save_state(path, dict(state, judged=[], learned=False, fallback_step=50))
    got, meta = load_state(path)
    assert got["judged"] == [] and got["learned"] is False and got["fallback_step"] == 50 and meta == {}
