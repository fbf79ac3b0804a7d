"""Shared test fixtures: the hand-derived closed-form cases and small helpers."""
import json
import os

import numpy as np

from paper_2103_01954_amd import scenes

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_closed_form():
    with open(os.path.join(GOLDEN, "closed_form_cases.json")) as f:
        return json.load(f)


def box_prims(boxes, M, half=0.25, bf16=False):
    n = len(boxes)
    pos = np.array([b["centre"] for b in boxes], dtype=np.float32).reshape(n, 3)
    rot = np.tile(np.eye(3, dtype=np.float32), (n, 1, 1))
    scale = np.full((n, 3), half, dtype=np.float32)
    pay = np.zeros((n, M, M, M, 4), dtype=np.float32)
    for k, b in enumerate(boxes):
        pay[k, ..., :3] = np.asarray(b["colour"], dtype=np.float32)
        pay[k, ..., 3] = np.float32(b["sigma"])
    if bf16:
        pay = scenes.bf16_round(pay)
    return scenes.Prims(pos, rot, scale, pay, bf16)


def closed_form_camera(spec):
    c = spec["camera"]
    return scenes.axis_camera(c["width"], c["height"], c["origin"], forward_axis=2, sign=-1.0,
                              focal=c["focal"])


def closed_form_case(spec, case):
    prims = box_prims(case["boxes"], spec["M"])
    cam = closed_form_camera(spec)
    params = scenes.MarchParams(case["step"], case["eps"])
    return prims, cam, params
