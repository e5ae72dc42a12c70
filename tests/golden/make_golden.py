"""Writes the regression fixtures of this folder from the FP64 oracle only.

    python tests/golden/make_golden.py

toy_paths.json     image-method paths of the toy workload (heuristic
                   candidates from 1e5 Fibonacci rays, one reflection):
                   per receiver the face sequences, coefficients a (re, im),
                   delays and angles.
toy_coverage.json  toy coverage map (1e5 rays, one reflection): total hits,
                   cells with hits, and the gain of 12 fixed cells.

The paper prints no worked numbers; these fixtures only freeze the oracle's
present output so that a change to its arithmetic is noticed (tests/
test_golden.py) and has to be justified.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import scenegen as sg  # noqa: E402
from oracle import geom, image, sbr  # noqa: E402

CELLS = [(100, 100), (100, 110), (120, 90), (60, 140), (150, 150), (30, 40), (100, 60), (80, 100), (130, 100),
         (101, 99), (170, 20), (10, 190)]


def toy_paths():
    w = sg.toy_workload()
    g = geom.Geometry(w.scene)
    r = sbr.trace(w.scene, w.tx[0], sbr.TraceParams(w.num_rays, w.max_depth), candidates=True, geo=g)
    P = image.paths(g, w.tx[0], w.rx, r.candidates)
    return {"candidates": sorted(list(c) for c in r.candidates),
            "rx": [[{"faces": list(p.faces), "a": [p.a.real, p.a.imag], "tau": p.tau, "aod": list(p.aod),
                     "aoa": list(p.aoa)} for p in pl] for pl in P]}


def toy_coverage():
    w = sg.toy_workload()
    gain, hits, namb = sbr.coverage(w.scene, w.tx[0], sbr.TraceParams(w.num_rays, w.max_depth), w.grid)
    return {"total_hits": int(hits.sum()), "cells_with_hits": int((hits > 0).sum()), "ambiguous_rays": namb,
            "cells": [[ix, iy, float(gain[iy, ix]), int(hits[iy, ix])] for ix, iy in CELLS]}


if __name__ == "__main__":
    with open(os.path.join(HERE, "toy_paths.json"), "w") as f:
        json.dump(toy_paths(), f, indent=1)
    with open(os.path.join(HERE, "toy_coverage.json"), "w") as f:
        json.dump(toy_coverage(), f, indent=1)
    print("written")
