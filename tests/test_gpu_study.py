"""The generalization study of the probed inverse (Rn preconditioners), on the GPU path."""
import numpy as np
import pytest

import fixtures as F

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_generalization_properties():
    """Along a nested chain of the paper's bases the fit residual never grows (a least-squares
    property), and the fitted inverse reconstructs an independent trial function from its
    image better than doing nothing (relative MSE below 1).  The MSE values themselves are
    not compared with the paper's (Marmousi) curves."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_3615_amd as M
    from paper_1101_3615_amd.study import generalization, paper_bases
    w = F.c1().with_(nt=400)
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c))
    trials = [torch.from_numpy(F.wavepackets(w, c, 200 + s, w.packets_per_trial)) for s in range(3)]
    bases = paper_bases(2, [(0, 0, 0), (0, 1, 1), (0, 2, 2), (1, 2, 2)])
    res = generalization(P, bases, trials[:2], trials[2])
    assert [r[0] for r in res] == [1, 4, 9, 63]
    relres = [r[2] for r in res]
    assert all(b <= a * (1 + 1e-9) for a, b in zip(relres, relres[1:])), relres
    assert all(not r[3] for r in res)
    assert min(r[1] for r in res) < 1.0
