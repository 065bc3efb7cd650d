"""The autotuner's cache (LBF_TUNE_CACHE): a workload tuned once is applied
from the file the next time, for single lattices and ensembles, and a
different workload is tuned afresh."""
import json

import pytest

import paper_0707_1581_amd as lbf

pytestmark = pytest.mark.gpu

BASE = dict(rho0=1.0, kT=1e-4, gamma_bulk=0.5, gamma_shear=0.8, gamma_odd=0.0, gamma_even=0.0)


def test_autotune_cache(tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("LBF_TUNE_CACHE", str(path))
    a = lbf.Lattice(48, 40, 36, **BASE, seed=1, init="thermal")
    ra = json.loads(a.autotune(steps=4))
    assert not any(r.get("cached") for r in ra)
    assert len(path.read_text().splitlines()) == 1
    b = lbf.Lattice(48, 40, 36, **BASE, seed=2, init="thermal")  # same workload, other seed
    rb = json.loads(b.autotune(steps=4))
    assert rb[0]["cached"] is True and rb[0]["key"] == path.read_text().split("\t")[0]
    assert b.schedule() == a.schedule()
    c = lbf.Lattice(40, 40, 36, **BASE, seed=1, init="thermal")  # another box: tuned afresh
    rc = json.loads(c.autotune(steps=4))
    assert not any(r.get("cached") for r in rc)
    assert len(path.read_text().splitlines()) == 2
    reps = [dict(BASE, nx=24, ny=20, nz=16, seed=s) for s in range(3)]
    e1 = lbf.Ensemble(reps, init="thermal")
    assert not any(r.get("cached") for r in json.loads(e1.autotune(steps=4)))
    e2 = lbf.Ensemble([dict(r, seed=r["seed"] + 10) for r in reps], init="thermal")
    assert json.loads(e2.autotune(steps=4))[0]["cached"] is True
    assert e2.schedule() == e1.schedule()
    b.step(6)  # the cached schedule runs
    assert b.check()[0] == 0
    for lat in (a, b, c, e1, e2):
        lat.close()


def test_autotune_cache_unwritable(tmp_path, monkeypatch):
    monkeypatch.setenv("LBF_TUNE_CACHE", str(tmp_path / "missing_dir" / "tune.txt"))
    a = lbf.Lattice(32, 32, 32, **BASE, seed=1, init="thermal")
    r = json.loads(a.autotune(steps=4))
    assert not any(x.get("cached") for x in r)
    a.step(4)
    assert a.check()[0] == 0
    a.close()


def test_autotune_cache_ignores_malformed_lines(tmp_path, monkeypatch):
    """Lines that are not `key<TAB>ten integers` are skipped: a matching key
    with a malformed schedule is tuned afresh, and the tuned line appended
    after it is used from then on."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("LBF_TUNE_CACHE", str(path))
    a = lbf.Lattice(40, 36, 32, **BASE, seed=1, init="thermal")
    a.autotune(steps=4)
    key = path.read_text().split("\t")[0]
    path.write_text("garbage without a tab\n" + key + "\t256 0 16\n" + "\t\n")
    b = lbf.Lattice(40, 36, 32, **BASE, seed=2, init="thermal")
    rb = json.loads(b.autotune(steps=4))
    assert not any(r.get("cached") for r in rb)
    lines = path.read_text().splitlines()
    assert len(lines) == 4 and lines[-1].startswith(key + "\t")
    c = lbf.Lattice(40, 36, 32, **BASE, seed=3, init="thermal")
    assert json.loads(c.autotune(steps=4))[0]["cached"] is True
    assert c.schedule() == b.schedule()
    for lat in (a, b, c):
        lat.close()
