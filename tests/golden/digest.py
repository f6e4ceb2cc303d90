"""Digests of reaction-step results, shared by the script that writes the
stored oracle digests (make_digests.py) and the GPU tests that compare the
library's results with them.  Hashing only: nothing here computes any part
of the reaction step.

A bond log is an int32 array of (step, id_A, id_T) rows, ordered by step and,
within a step, by id_A.  A step's digest is the first 16 hex digits of the
SHA-256 of its rows' little-endian int32 bytes; an array digest that of the
array's bytes (C order, little-endian)."""
import hashlib

import numpy as np

STAT_NAMES = ("a_elig", "t_elig", "in_rc", "drawn", "excluded", "accepted", "proposals", "bonds",
              "adj_overflow")


def h16(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).astype(np.asarray(a).dtype.newbyteorder("<"),
                                                copy=False).tobytes())
    return h.hexdigest()[:16]


def step_digests(log, first, n_steps):
    """{step: (bond count, digest)} for steps first .. first + n_steps - 1."""
    log = np.ascontiguousarray(log, dtype=np.int32).reshape(-1, 3)
    out = {}
    steps = log[:, 0]
    lo = np.searchsorted(steps, np.arange(first, first + n_steps), side="left")
    hi = np.searchsorted(steps, np.arange(first, first + n_steps), side="right")
    for k in range(n_steps):
        rows = log[lo[k]:hi[k]]
        out[first + k] = (int(rows.shape[0]), h16(rows))
    return out


def config_digests(x, y, z, state, adj):
    """Digests of a final configuration in particle-id order."""
    return {"pos": h16(np.asarray(x, np.float32), np.asarray(y, np.float32),
                       np.asarray(z, np.float32)),
            "state": h16(np.asarray(state, np.int32)), "adj": h16(np.asarray(adj, np.int32))}


def write_traj(path, header, per_step, final):
    """per_step: list of (step, stats tuple of 9, digest); final: dict."""
    with open(path, "w") as f:
        for line in header:
            f.write("# %s\n" % line)
        f.write("# columns: step %s bonds_sha16\n" % " ".join(STAT_NAMES))
        for step, st, dg in per_step:
            f.write("%d %s %s\n" % (step, " ".join(str(int(v)) for v in st), dg))
        f.write("final pos=%s state=%s adj=%s\n" % (final["pos"], final["state"], final["adj"]))


def read_traj(path):
    """(header lines, {step: (stats tuple, digest)}, final dict)."""
    header, steps, final = [], {}, None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                header.append(line[1:].strip())
            elif line.startswith("final"):
                final = dict(kv.split("=") for kv in line.split()[1:])
            else:
                p = line.split()
                steps[int(p[0])] = (tuple(int(v) for v in p[1:10]), p[10])
    return header, steps, final
