"""Checkpoint files of the learned-preconditioner training (host logic only)."""
import numpy as np
import pytest

from paper_2011_01850_amd import train as T


class FakeOpt:
    def __init__(self, seed):
        g = np.random.default_rng(seed)
        self.st = {"theta": g.standard_normal(9665).astype(np.float32),
                   "m1": g.standard_normal(9665).astype(np.float32),
                   "m2": np.abs(g.standard_normal(9665)).astype(np.float32),
                   "t": 17, "lr": 1e-3, "beta1": 0.9, "beta2": 0.999, "eps": 1e-8}

    def state_dict(self):
        return self.st


def test_checkpoint_round_trip(tmp_path):
    path = str(tmp_path / "ck.npz")
    opt = FakeOpt(3)
    T.save_checkpoint(path, opt, 42, [0.5, 0.25, 0.125], seed=7, ninst=2000, batch=4)
    ck = T.load_checkpoint(path)
    assert (ck["step"], ck["seed"], ck["ninst"], ck["batch"]) == (42, 7, 2000, 4)
    assert ck["history"] == [0.5, 0.25, 0.125]
    for name in ("theta", "m1", "m2"):
        assert ck["opt"][name].dtype == np.float32
        assert np.array_equal(ck["opt"][name], opt.st[name])
    for name in ("t", "lr", "beta1", "beta2", "eps"):
        assert ck["opt"][name] == opt.st[name]
    # an overwrite replaces the file whole
    T.save_checkpoint(path, FakeOpt(4), 43, [1.0], seed=7, ninst=2000, batch=4)
    assert T.load_checkpoint(path)["step"] == 43


def test_checkpoint_needs_no_pickle(tmp_path):
    path = str(tmp_path / "ck.npz")
    T.save_checkpoint(path, FakeOpt(1), 1, [], seed=0, ninst=1, batch=1)
    with np.load(path, allow_pickle=False) as z:
        assert all(z[k].dtype != object for k in z.files)
    with pytest.raises(FileNotFoundError):
        T.load_checkpoint(str(tmp_path / "missing.npz"))
