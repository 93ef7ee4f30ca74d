"""The launch-shape tuning table (host code only, no device calls): defaults,
set/get, the JSON cache round trip, and rejection of malformed files."""
import json
import os

import pytest

import paper_1905_06706_amd as hg


@pytest.fixture()
def lib(monkeypatch):
    monkeypatch.delenv("GIRG_BATCH_WORKERS", raising=False)
    try:
        hg.load()
    except ImportError as e:
        pytest.skip(str(e))
    hg.tuning_reset()
    yield hg
    hg.tuning_reset()


def test_defaults(lib):
    assert lib.tuning_get(lib.make_params(10**4, 1, 2.5, 0.0, 10.0)) == (512, 16)
    assert lib.tuning_get(lib.make_params(2**17 - 1, 1, 2.5, 0.0, 10.0))[0] == 512
    assert lib.tuning_get(lib.make_params(2**17, 1, 2.5, 0.0, 10.0))[0] == 1024
    assert lib.tuning_get(lib.make_params(2**20, 3, 2.5, 0.0, 10.0))[0] == 1024
    assert lib.tuning_get(lib.make_params(2**22 - 1, 2, 2.7, 0.5, 16.0))[0] == 512
    assert lib.tuning_get(lib.make_params(2**22, 2, 2.7, 0.5, 16.0))[0] == 1024
    assert lib.tuning_get(lib.make_params(2**21, 3, 2.3, 0.8, 20.0))[0] == 768
    assert lib.tuning_get(lib.make_params(2**19, 4, 2.5, 0.5, 10.0))[0] == 768
    assert lib.tuning_get(lib.make_params(2**18 - 1, 3, 2.5, 0.5, 16.0))[0] == 512
    assert lib.tuning_get(lib.make_params(2**18, 3, 2.5, 0.5, 16.0))[0] == 768
    assert lib.tuning_get(lib.make_params(2**17 - 1, 2, 2.7, 0.5, 16.0))[0] == 256
    assert lib.tuning_get(lib.make_params(2**17, 2, 2.7, 0.5, 16.0))[0] == 512
    assert lib.tuning_get(lib.make_params(2**16, 3, 2.5, 0.5, 16.0))[0] == 512
    assert lib.tuning_get(lib.make_params(2**22, 3, 2.3, 0.8, 20.0))[0] == 1024
    assert lib.tuning_get(lib.make_params(10**7, 3, 2.3, 0.8, 20.0))[0] == 1024
    assert lib.tuning_get(lib.make_params(10**4, 1, 2.5, 0.0, 10.0), batch=True) == (256, 16)


def test_set_get_by_class(lib):
    p = lib.make_params(2**20, 2, 2.7, 0.5, 16.0)
    lib.tuning_set(p, 2048)
    assert lib.tuning_get(p)[0] == 2048
    # same class: floor(log2 n), d, T > 0, model
    assert lib.tuning_get(lib.make_params(2**21 - 1, 2, 2.1, 0.9, 8.0))[0] == 2048
    assert lib.tuning_get(lib.make_params(2**21, 2, 2.7, 0.5, 16.0))[0] == 512
    assert lib.tuning_get(lib.make_params(2**20, 2, 2.7, 0.0, 16.0))[0] == 1024
    assert lib.tuning_get(lib.make_params(2**20, 3, 2.7, 0.5, 16.0))[0] == 768
    h = lib.make_params(2**20, 1, 0.0, 0.5, 10.0, model=1, alpha=0.75)
    assert lib.tuning_get(h)[0] == 512
    lib.tuning_set(h, 768)
    assert lib.tuning_get(h)[0] == 768
    assert lib.tuning_get(lib.make_params(2**20, 1, 2.5, 0.5, 10.0))[0] == 512
    lib.tuning_set(None, 256, batch=True, workers=8)
    assert lib.tuning_get(p, batch=True) == (256, 8)
    lib.tuning_set(None, 384, batch=True)  # workers 0 keeps 8
    assert lib.tuning_get(p, batch=True) == (384, 8)


def test_env_overrides_batch_workers(lib, monkeypatch):
    monkeypatch.setenv("GIRG_BATCH_WORKERS", "5")
    assert lib.tuning_get(lib.make_params(1000, 1, 2.5, 0.0, 10.0), batch=True)[1] == 5


def test_invalid_values(lib):
    p = lib.make_params(2**20, 2, 2.7, 0.5, 16.0)
    for blocks in (0, -3, 8193):
        with pytest.raises(lib.GirgError):
            lib.tuning_set(p, blocks)
    with pytest.raises(lib.GirgError):
        lib.tuning_set(None, 512, batch=True, workers=65)
    with pytest.raises(lib.GirgError):
        lib.tuning_set(lib.make_params(2**20, 5, 2.7, 0.5, 16.0), 512)
    assert lib.tuning_get(p)[0] == 512


def test_save_load_round_trip(lib, tmp_path):
    p1 = lib.make_params(2**20, 2, 2.7, 0.5, 16.0)
    p2 = lib.make_params(10**4, 1, 2.5, 0.0, 10.0)
    p3 = lib.make_params(2**20, 1, 0.0, 0.5, 10.0, model=1, alpha=0.75)
    lib.tuning_set(p1, 1536)
    lib.tuning_set(p2, 256)
    lib.tuning_set(p3, 768)
    lib.tuning_set(None, 768, batch=True, workers=12)
    path = str(tmp_path / "tune.json")
    lib.tuning_save(path)
    doc = json.load(open(path))
    assert doc["version"] == 1
    assert doc["batch"] == {"blocks": 768, "workers": 12}
    assert {"model": 0, "d": 2, "binomial": 1, "log2n": 20, "blocks": 1536} in doc["single"]
    assert {"model": 0, "d": 1, "binomial": 0, "log2n": 13, "blocks": 256} in doc["single"]
    assert {"model": 1, "d": 1, "binomial": 1, "log2n": 20, "blocks": 768} in doc["single"]
    lib.tuning_reset()
    assert lib.tuning_get(p1)[0] == 512
    lib.tuning_load(path)
    assert lib.tuning_get(p1)[0] == 1536
    assert lib.tuning_get(p2)[0] == 256
    assert lib.tuning_get(p3)[0] == 768
    assert lib.tuning_get(p1, batch=True) == (768, 12)


@pytest.mark.parametrize("text", [
    "",
    "{",
    '{"version": 2, "single": []}',
    '{"version": 1, "single": [{"model": 0, "d": 2, "binomial": 1, "log2n": 20}]}',
    '{"version": 1, "single": [{"model": 0, "d": 9, "binomial": 1, "log2n": 20, "blocks": 64}]}',
    '{"version": 1, "single": [{"model": 0, "d": 2, "binomial": 1, "log2n": 20, "blocks": 0}]}',
    '{"version": 1, "single": [{"model": 0, "d": 2, "binomial": 1, "log2n": 20, "blocks": 6.5}]}',
    '{"version": 1, "batch": {"blocks": 512, "workers": 0}}',
    '{"version": 1, "batch": {"blocks": 512}}',
    '{"version": 1, "extra": 3}',
    '{"version": 1, "batch": {"blocks": -}}',
    '{"version": 1, "single": [{"model": 0, "d": 2, "binomial": 1, "log2n": 20, "blocks": 64}',
    'not json',
])
def test_malformed_files_leave_table(lib, tmp_path, text):
    p = lib.make_params(2**20, 2, 2.7, 0.5, 16.0)
    lib.tuning_set(p, 1536)
    path = tmp_path / "bad.json"
    path.write_text(text)
    with pytest.raises(lib.GirgError) as ei:
        lib.tuning_load(str(path))
    assert ei.value.status == lib.GIRG_EINVAL
    assert lib.tuning_get(p)[0] == 1536


def test_missing_file(lib, tmp_path):
    with pytest.raises(lib.GirgError):
        lib.tuning_load(str(tmp_path / "nope.json"))
    with pytest.raises(lib.GirgError):
        lib.tuning_save(os.path.join(str(tmp_path), "no_dir", "x.json"))


def test_env_tuning_file_loaded_at_first_call(tmp_path):
    """GIRG_TUNING_FILE is read once, at the library's first tuning lookup (a
    fresh process); a malformed file is reported on stderr and ignored."""
    import subprocess
    import sys
    good = tmp_path / "good.json"
    good.write_text('{"version": 1, "single": [{"model": 0, "d": 2, "binomial": 1, "log2n": 20, '
                    '"blocks": 640}], "batch": {"blocks": 320, "workers": 6}}')
    bad = tmp_path / "bad.json"
    bad.write_text('{"version": 1, "single": [{"model": 0}]}')
    code = ("import paper_1905_06706_amd as hg\n"
            "p = hg.make_params(2**20, 2, 2.7, 0.5, 16.0)\n"
            "print(hg.tuning_get(p)[0], *hg.tuning_get(p, batch=True))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, GIRG_TUNING_FILE=str(good))
    env.pop("GIRG_BATCH_WORKERS", None)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.split() == ["640", "320", "6"]
    env["GIRG_TUNING_FILE"] = str(bad)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.split() == ["512", "256", "16"]
    assert "GIRG_TUNING_FILE ignored" in r.stderr
