"""The oracle's command line (python -m oracle) gives what its Python API gives."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _cli(*args):
    subprocess.run([sys.executable, "-m", "oracle", *args], cwd=ROOT, check=True, capture_output=True)


def test_cli_matches_api(orc, tmp_path):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((400, 4)).astype(np.float32)
    ell = np.array([0.7, 1.0, 1.3, 0.9])
    V = rng.standard_normal((400, 2))
    p = {k: str(tmp_path / f"{k}.npy") for k in ("X", "ell", "V")}
    np.save(p["X"], X)
    np.save(p["ell"], ell)
    np.save(p["V"], V)
    lat = orc.Lattice(X, ell)

    _cli("build", "--X", p["X"], "--ell", p["ell"], "--out", str(tmp_path / "lat"))
    for name, ref in zip(("keys", "idx", "w", "nbr"), lat.export()):
        np.testing.assert_array_equal(np.load(tmp_path / f"lat_{name}.npy"), ref)

    _cli("mvm", "--X", p["X"], "--ell", p["ell"], "--values", p["V"], "--outputscale", "1.5",
         "--out", str(tmp_path / "y.npy"))
    np.testing.assert_array_equal(np.load(tmp_path / "y.npy"), lat.mvm(V, outputscale=1.5))

    _cli("cg", "--X", p["X"], "--ell", p["ell"], "--values", p["V"], "--noise", "0.2", "--tol", "1e-6",
         "--out", str(tmp_path / "x.npy"))
    np.testing.assert_array_equal(np.load(tmp_path / "x.npy"), lat.cg(V, 0.2, 1e-6)[0])
