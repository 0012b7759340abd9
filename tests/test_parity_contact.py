"""The parity contract's treatment of agents in contact within rounding
(CPU): a pair whose FP64 gap is +5e-10 m, while the FP32 contact test
finds |P|^2 == R^2 and takes the overlap form of the velocity obstacle."""
import dataclasses

import numpy as np

import oracle
from paper_2008_11578_amd import scenarios

from parity import V_TOL, contact_flipped

F32 = np.float32


def _pair(dx=0.0):
    # positions and velocities of a touching pair met in the dense crossing
    # (the FP64 gap is 4.97e-10 m; in FP32 the squared distance rounds to
    # R^2 exactly); the first agent's goal lies beyond the second, so that
    # their constraint binds
    px = np.array([596.8102, 597.1426 + dx], F32)
    py = np.array([448.89795, 448.39844], F32)
    P = (float(px[1]) - float(px[0]), float(py[1]) - float(py[0]))
    st = dict(px=px, py=py,
              vx=np.array([-0.55613786, -0.767137], F32), vy=np.array([-0.042509288, -0.18403682], F32),
              pref_x=np.array([float(px[0]) + 100 * P[0], 101.54251], F32),
              pref_y=np.array([float(py[0]) + 100 * P[1], 448.7791], F32),
              radius=np.full(2, 0.3, F32), max_speed=np.full(2, 1.5, F32), cls=np.zeros(2, np.uint8))
    return st


def _params():
    return dataclasses.replace(scenarios.c3_crossing(side_count=4).params, cell_size=0.6)


def test_pair_is_a_contact_within_rounding():
    st = _pair()
    P = np.array([st["px"][1] - st["px"][0], st["py"][1] - st["py"][0]], F32)
    R = F32(st["radius"][0] + st["radius"][1])
    assert not (F32(P[0] * P[0] + P[1] * P[1]) > F32(R * R))            # FP32: overlap
    d = np.hypot(float(st["px"][1]) - float(st["px"][0]), float(st["py"][1]) - float(st["py"][0]))
    assert 0.0 < d - 0.6000000238418579 < 1e-9                          # FP64: apart


def test_contact_flip_accepts_only_the_other_side():
    st, p = _pair(), _params()
    o = oracle.step(st, p)
    r = st["radius"].copy()
    r[0] = np.nextafter(r[0], F32(np.inf))
    flipped = oracle.step(dict(st, radius=r), p)
    # the two sides of the contact give different answers
    assert np.hypot(o["vx"][0] - flipped["vx"][0], o["vy"][0] - flipped["vy"][0]) > V_TOL
    g = {k: flipped[k] for k in ("vx", "vy")}
    assert contact_flipped(st, p, 0, g)
    # an answer that matches neither side is refused
    g_bad = {"vx": flipped["vx"] + 10 * V_TOL, "vy": flipped["vy"]}
    assert not contact_flipped(st, p, 0, g_bad)
    # agents 1 mm apart are no contact within rounding
    assert not contact_flipped(_pair(dx=0.001), p, 0, g)
