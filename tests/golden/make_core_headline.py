"""Writes core_headline_256.json: what the float64 oracle's Core Stage gives on
the 256^2 problem of the full-size Core Stage GPU test (53,856 samples of the
Lissajous figure, cosine interpolation, window 31, gamma = 1e-3, tol = 1e-3,
inputs rounded to float32).  Calls only the oracle and the input generators;
about 90 s.  Run from the repository root:
    python tests/golden/make_core_headline.py
"""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
import oracle as O                                        # noqa: E402
from paper_2505_22797_amd import synth as S               # noqa: E402


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def main():
    P = S.headline()
    n, t, R, gamma, tol, seed = P.n, P.n_samples, 31, 1e-3, 1e-3, 5
    tr = S.lissajous(t, ax=0.85, ay=0.85)
    r, v = f32(tr.r), f32(tr.v)
    h = S.h_fwhm2(n)
    c = S.ellipses_and_line(n, seed)
    M = O.Model(n, h, R, r, v, interp="cosine")
    s = f32(S.add_noise(M.forward(c), 30.0, seed=seed))
    a, steps = O.core_stage(s, r, v, n, gamma, tol=tol, max_iter=10000)
    b = O.core_rhs(s, r, v, n)
    G = M.field(c)
    out = dict(n=n, n_samples=t, radius=R, gamma=gamma, tol=tol, seed=seed, steps=int(steps),
               true_residual=float(np.linalg.norm(O.core_normal(a, r, v, gamma) - b) / np.linalg.norm(b)),
               field_error=float(np.linalg.norm(a - G) / np.linalg.norm(G)))
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "core_headline_256.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(out)


if __name__ == "__main__":
    main()
