"""What the trained surrogate gains over the method without it: on held-out static-tissue
samples, the ADE-only iteration started from the network's prediction reaches the same
stopping rule (relative change 1e-6) in fewer iterations than from zero, and both end within
the error the rule allows of each other."""
import sys

import numpy as np
import pytest

from paper_1503_06726_amd import lbib
from paper_1503_06726_amd import warmstart as WS

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_trained_warm_start_needs_fewer_iterations():
    ws = WS.generate(range(32), held_out=True, workers=1)
    src, _, feat = WS.prepare(ws)
    k0, phi0 = WS.solve(ws, src, tol=1e-6)
    params, meta = WS.load()
    net = lbib.Net(ws[0].ny, ws[0].nx, 16)
    net.set_params(params)
    phi_hat = WS.predict(net, feat, ws)
    net.close()
    kw, phiw = WS.solve(ws, src, phi0=phi_hat, tol=1e-6)
    say(f"  32 held-out samples: zero start median {np.median(k0):.0f} mean {k0.mean():.0f}; "
        f"warm start median {np.median(kw):.0f} mean {kw.mean():.0f} (trained on {meta['samples']} samples)")
    assert (k0 > 0).all() and (kw > 0).all()
    assert np.median(kw) <= 0.6 * np.median(k0) and kw.mean() <= 0.6 * k0.mean()
    # both runs stop within about tol / decay of the steady state
    for i, w in enumerate(ws):
        lam = w.species[0].c[1]
        d = np.linalg.norm(phiw[i] - phi0[i]) / np.linalg.norm(phi0[i])
        assert d <= 4e-6 / lam, (i, d, lam)
