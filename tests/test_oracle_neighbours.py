"""Pin of the oracle's cell-list pair set against brute force."""
import numpy as np
import pytest

import synth
from oracle import oracle as O


def brute(X, box, rc, periodic_y=True):
    n = len(X)
    out = []
    for i in range(n):
        d = X[i + 1:] - X[i]
        for a in range(3):
            if a == 1 and not periodic_y:
                continue
            L = box[a]
            d[:, a] = np.where(d[:, a] >= 0.5 * L, d[:, a] - L, np.where(d[:, a] < -0.5 * L, d[:, a] + L, d[:, a]))
        r2 = (d ** 2).sum(1)
        for j in np.nonzero(r2 < rc * rc)[0]:
            out.append((i, i + 1 + j))
    return np.array(out, dtype=np.int32).reshape(-1, 2)


@pytest.mark.parametrize("box,N,rc,walls", [((32, 32, 32), 400, 3.75, 0), ((24, 24, 48), 300, 5.45, 1),
                                             ((8, 9, 10), 40, 3.75, 0), ((12, 12, 12), 80, 5.0, 0)])
def test_pairs_match_bruteforce(box, N, rc, walls):
    rng = np.random.default_rng(N)
    p = synth.params(*box, wall_y=walls, r_cut=rc)
    X = rng.random((N, 3)) * box
    if walls:
        X[:, 1] = 1 + rng.random(N) * (box[1] - 2)
    o = O.Oracle(p)
    o.set_particles(X, synth.random_quaternions(rng, N), fixed=np.ones(N, np.uint8))
    got = o.pairs()
    want = brute(X, box, rc, periodic_y=not walls)
    assert got.shape == want.shape and (got == want).all()
