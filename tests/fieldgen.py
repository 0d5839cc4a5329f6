"""Gauge fields for GPU tests, drawn in a child Python process that never touches the GPU.

lattice_inputs.random_gauges forks worker processes, which a process that has
initialised a GPU must not do; the child draws the fields (the same seeded
streams as the serial calls) and hands them back through .npy files.
"""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_CHILD = """
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import lattice_inputs as li
jobs = [(tuple(j[0]), j[1], j[2]) for j in json.loads(sys.argv[2])]
for k, u in enumerate(li.random_gauges(jobs)):
    np.save(f"{sys.argv[3]}/field{k}.npy", u)
"""


def random_gauges_in_child(jobs, tmpdir, timeout=600):
    """li.random_gauge(L, eps, seed) for each job, computed in a child process."""
    spec = json.dumps([[list(L), float(eps), int(seed)] for L, eps, seed in jobs])
    subprocess.run([sys.executable, "-c", _CHILD, ROOT, spec, str(tmpdir)], check=True, timeout=timeout)
    out = []
    for k in range(len(jobs)):
        path = os.path.join(str(tmpdir), f"field{k}.npy")
        out.append(np.load(path))
        os.remove(path)
    return out
