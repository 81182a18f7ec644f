"""Helpers for the GPU parity tests: oracle plans on the golden placements
and host/device conversion.  No transform arithmetic here."""

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_theta(L):
    path = os.path.join(GOLDEN, f"theta_greedy_L{L}.txt")
    if not os.path.exists(path):
        return None
    return np.asarray([int(x) for x in open(path) if not x.startswith("#")])


def oracle_plan(L, s=0, placement="greedy"):
    from oracle import sht
    num = golden_theta(L) if placement == "greedy" else None
    return sht.Plan(L, s, numerators=num, placement=placement)


def to_dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.complex128)).cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relmax(a, b):
    b = np.asarray(b)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(np.asarray(a) - b)) / (den if den > 0 else 1.0))


def read_golden_values(name):
    """(header dict, rows) of a tests/golden value file: '# key value' header
    lines (max_abs is parsed as a float), then whitespace-separated rows whose
    last two columns are the real and imaginary parts."""
    head, rows = {}, []
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#"):
            parts = line[1:].split()
            if len(parts) == 2 and parts[0] == "max_abs":
                head["max_abs"] = float(parts[1])
            continue
        rows.append(line.split())
    return head, rows
