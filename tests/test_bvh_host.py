"""Host build of the scene preparation code (C++, compiled with g++ here):
BVH structure invariants, face grouping equal to the oracle's, and closest
hits through the BVH equal to the brute-force oracle."""
import os
import subprocess

import numpy as np
import pytest

import scenegen as sg
from oracle import geom, native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_11103_amd", "csrc")


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("bvh_host"))


@pytest.fixture(scope="module")
def checker(workdir):
    exe = os.path.join(workdir, "bvh_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, os.path.join(CSRC, "scene.cpp"),
                    os.path.join(ROOT, "tests", "host", "bvh_check.cpp"), "-o", exe], check=True)
    return exe


def _run(exe, s, O, D):
    work = os.path.dirname(exe)
    inp = os.path.join(work, "bvh_in.bin")
    out = os.path.join(work, "bvh_out.bin")
    with open(inp, "wb") as f:
        np.asarray([len(s.V), s.nt, len(s.materials), len(O)], dtype=np.int64).tofile(f)
        np.ascontiguousarray(s.V, dtype=np.float32).tofile(f)
        np.ascontiguousarray(s.F, dtype=np.int32).tofile(f)
        np.ascontiguousarray(s.tri_mat, dtype=np.int32).tofile(f)
        np.ascontiguousarray(O, dtype=np.float64).tofile(f)
        np.ascontiguousarray(D, dtype=np.float64).tofile(f)
    r = subprocess.run([exe, inp, out], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    raw = open(out, "rb").read()
    nt, nr = s.nt, len(O)
    faces = np.frombuffer(raw[:4 * nt], dtype=np.int32)
    hit = np.frombuffer(raw[4 * nt:4 * nt + 4 * nr], dtype=np.int32)
    off = 4 * nt + 4 * nr + 8 * nr
    t = np.frombuffer(raw[4 * nt + 4 * nr:off], dtype=np.float64)
    nw = int(np.frombuffer(raw[off:off + 4], dtype=np.int32)[0])
    wedges = np.frombuffer(raw[off + 4:], dtype=np.float64).reshape(nw, 16)
    return faces, hit, t, wedges, r.stdout


@pytest.mark.parametrize("name", ["toy", "urban", "city"])
def test_bvh_closest_hits_and_faces_match_oracle(checker, name):
    s = {"toy": sg.make_toy, "urban": lambda: sg.make_urban(0), "city": lambda: sg.make_city(0, blocks=10)}[name]()
    lo, hi = (-90, 90) if name == "toy" else (-230, 230) if name == "urban" else (-200, 200)
    O, D = sg.random_rays(3000, seed=3, lo=lo, hi=hi, zlo=0.5, zhi=80)
    faces, hit, t, _, _ = _run(checker, s, O, D)
    ref_faces, _ = geom.face_ids(s.V, s.F, s.tri_mat)
    assert np.array_equal(faces, ref_faces)
    g = geom.Geometry(s)
    tri, tt, margin = native.closest_hit(O, D, np.full(len(O), -1), 1e-4, g.V, g.F, g.face, want_margin=True)
    ok = margin >= 1e-6
    assert ok.mean() > 0.9  # origins inside buildings see floor/ground ties (margin 0)
    assert np.array_equal(hit[ok], tri[ok])
    h = ok & (tri >= 0)
    assert np.max(np.abs(t[h] - tt[h]) / (1 + tt[h])) < 1e-12


@pytest.mark.parametrize("name", ["toy", "urban", "city"])
def test_diffraction_wedges_match_oracle(checker, name):
    """The host extraction of diffraction wedges equals the oracle's: same
    wedges in the same order, same frames and exterior angles."""
    from oracle import diffraction
    s = {"toy": sg.make_toy, "urban": lambda: sg.make_urban(0), "city": lambda: sg.make_city(0, blocks=6)}[name]()
    O, D = sg.random_rays(4, seed=3, lo=-50, hi=50, zlo=0.5, zhi=80)
    _, _, _, wg, _ = _run(checker, s, O, D)
    ref = diffraction.wedges(geom.Geometry(s))
    assert len(ref) == wg.shape[0] > 0
    for w, r in zip(ref, wg):
        assert np.array_equal(w.a, r[0:3])
        assert np.allclose(w.e, r[3:6], atol=1e-15) and np.allclose(w.t0, r[6:9], atol=1e-15)
        assert np.allclose(w.n0, r[9:12], atol=1e-15)
        assert abs(w.length - r[12]) < 1e-12 * w.length and abs(w.n - r[13]) < 1e-14
        assert (w.face0, w.facen) == (int(r[14]), int(r[15]))


def test_ground_quad_leaf_sits_near_the_root(checker):
    """The size partition of the SAH build: the city's ground quad (input
    triangles 0 and 1, each with a box of the whole city's footprint) becomes
    a leaf within two levels of the root (a binned split alone carried it
    four levels down, widening the boxes of every node on the way)."""
    s = sg.make_city(0, blocks=10)
    O, D = sg.random_rays(4, seed=3, lo=-50, hi=50, zlo=0.5, zhi=80)
    *_, out = _run(checker, s, O, D)
    line = [l for l in out.splitlines() if l.startswith("leaf_depth_of_triangle_0")][0]
    assert 1 <= int(line.split()[1]) <= 2
