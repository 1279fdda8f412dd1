"""Host-side checks of bench.py's contract (no device work)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("mixed,fp32,per_cell", [(False, False, 1752), (True, False, 1552), (True, True, 928)])
def test_weno_algorithmic_bytes(mixed, fp32, per_cell):
    """Per-cell WENO bytes of the three precision forms: ids 64, state 40 (20 in FP32),
    pseudo-inverse 1152 (576), geometry 56 (28), centroid 24, image codes 16, record 400
    (200 in both reduced forms)."""
    assert bench.algorithmic_bytes("weno", 1000, 2000, mixed, fp32) == 1000 * per_cell


def test_flux_and_update_algorithmic_bytes():
    nc, nf = 1000, 2000
    # the mean of 216 (first stage) and 176 (second stage, dF only) per face
    assert bench.algorithmic_bytes("flux", nc, nf, False) == nf * 196 + nc * 400
    assert bench.algorithmic_bytes("update", nc, nf, False) == nc * 292
    # the FP32 form: 4-byte geometry, fluxes and state, 4-byte ids as before
    assert bench.algorithmic_bytes("flux", nc, nf, True, True) == nf * 102 + nc * 220
    assert bench.algorithmic_bytes("update", nc, nf, True, True) == nc * 154


def test_hex_weno_algorithmic_bytes():
    """Per hexahedral cell: 24 stencil ids (96), own state (40), the 9 x 24 pseudo-inverse
    (1728), eight 3 x 3 sub-stencil inverses (576), seven geometry values (56) and the
    record written: 400 B in FP64, 200 B in FP32-mixed."""
    assert bench.algorithmic_bytes("weno_hex", 1000, 0, False) == 1000 * 2896
    assert bench.algorithmic_bytes("weno_hex", 1000, 0, True) == 1000 * 2696

