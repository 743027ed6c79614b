"""CPU test of the conservative ellipse-rectangle test that the render kernels
use to skip (entry, pixel group) pairs and that tile culling uses to drop
pairs (msplat::ellipse_meets, compiled for the host from the same header the
kernels include).  Against brute-force enumeration of pixel centres: whenever
some pixel centre of the rectangle reaches alpha_min (evaluated in float32
exactly as the kernels do, and in float64), the test must say the ellipse
meets the rectangle, so culling never drops a pair that Eq. (1) composites;
and it must reject most rectangles the ellipse cannot reach."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LOG2E = 1.4426950408889634


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("em") / "ellipse_meets_host")
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "ellipse_meets_host.cpp"), "-o", exe])
    return exe


def _cases(seed, count):
    g = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        # a 2D Gaussian: covariance from random axes and angle (+ low-pass), opacity
        s1, s2 = np.exp(g.uniform(np.log(0.3), np.log(40.0), 2))
        th = g.uniform(0, np.pi)
        Rm = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        S = Rm @ np.diag([s1 * s1, s2 * s2]) @ Rm.T + 0.3 * np.eye(2)
        a, b, c = np.linalg.inv(S)[0, 0], np.linalg.inv(S)[0, 1], np.linalg.inv(S)[1, 1]
        o = g.uniform(1 / 255, 1.0)
        u, v = g.uniform(100, 200, 2)
        uh, vh = np.float32(u), np.float32(v)
        rec = [uh, vh, np.float32(u - float(uh)), np.float32(v - float(vh)), np.float32(0.5 * LOG2E * a),
               np.float32(LOG2E * b), np.float32(0.5 * LOG2E * c), np.float32(np.log2(o))]
        # rectangles near the alpha_min ellipse: inside its bounding box, on
        # its edge or just outside, where a box test alone keeps them
        ext = np.sqrt(max(2.0 * np.log(255.0 * o), 1e-9) * np.diag(S))
        w, h = g.integers(0, 16, 2)
        cx, cy = u + g.uniform(-1.3, 1.3) * ext[0], v + g.uniform(-1.3, 1.3) * ext[1]
        x0, y0 = int(np.floor(cx - w / 2)), int(np.floor(cy - h / 2))
        x1, y1 = x0 + int(w), y0 + int(h)
        out.append((rec, int(x0), int(x1), int(y0), int(y1)))
    return out


def _reachable(rec, x0, x1, y0, y1, la):
    """Largest exponent over the rectangle's pixel centres: float32 as the kernels, and float64."""
    f = np.float32
    xs = np.arange(x0, x1 + 1, dtype=np.float32) + f(0.5)
    ys = np.arange(y0, y1 + 1, dtype=np.float32) + f(0.5)
    X, Y = np.meshgrid(xs, ys)
    dx = (X - rec[0]) - rec[2]
    dy = (Y - rec[1]) - rec[3]
    ee32 = rec[7] - (rec[4] * dx * dx + rec[5] * dx * dy + rec[6] * dy * dy)
    dx64 = X.astype(np.float64) - (float(rec[0]) + float(rec[2]))
    dy64 = Y.astype(np.float64) - (float(rec[1]) + float(rec[3]))
    ee64 = float(rec[7]) - (float(rec[4]) * dx64 ** 2 + float(rec[5]) * dx64 * dy64 + float(rec[6]) * dy64 ** 2)
    return bool((ee32 >= f(la)).any()), float(ee64.max())


def test_ellipse_meets_is_conservative_and_useful(driver):
    la = float(np.float32(np.log2(np.float32(1.0 / 255.0))))
    cases = _cases(1, 6000)
    lines = []
    for rec, x0, x1, y0, y1 in cases:
        lines.append(" ".join(float(x).hex() for x in rec) + f" {x0} {x1} {y0} {y1} {float(np.float32(la)).hex()}")
    res = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    got = [int(x) for x in res.stdout.split()]
    assert len(got) == len(cases)
    reach = cut = 0
    for (rec, x0, x1, y0, y1), meets in zip(cases, got):
        hit32, e64 = _reachable(rec, x0, x1, y0, y1, la)
        if hit32 or e64 >= la:
            reach += 1
            assert meets == 1, (rec, x0, x1, y0, y1)
        elif meets == 0:
            cut += 1
    unreachable = len(cases) - reach
    assert reach > 1000 and unreachable > 1000
    # most unreachable rectangles near the ellipse are rejected
    assert cut > 0.8 * unreachable, (cut, unreachable)
