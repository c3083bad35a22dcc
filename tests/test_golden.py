"""The closed-form fixtures under tests/golden/ checked from first principles:
the coordination shells of FCC and BCC by enumerating lattice points."""
import json
import os
from collections import Counter

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def shells(basis, nshell):
    """Squared distance / a^2 and multiplicity of the first shells around a
    lattice site, by brute force over the conventional cells around it."""
    g = np.arange(-3, 4)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pts = (cells[:, None, :] + np.asarray(basis)[None, :, :]).reshape(-1, 3)
    d2 = np.round((pts ** 2).sum(1) * 4).astype(int)  # 4 r^2 / a^2 is an integer for both
    c = Counter(d2[d2 > 0].tolist())
    keys = sorted(c)[:nshell]
    return [k / 4 for k in keys], [c[k] for k in keys]


def test_lattice_shells_fixture():
    fx = json.load(open(os.path.join(HERE, "golden", "lattice_shells.json")))
    fcc = [[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]
    bcc = [[0, 0, 0], [0.5, 0.5, 0.5]]
    for name, basis in (("fcc", fcc), ("bcc", bcc)):
        n = len(fx[name]["count"])
        r2, cnt = shells(basis, n)
        assert r2 == fx[name]["r_over_a_squared"], name
        assert cnt == fx[name]["count"], name
