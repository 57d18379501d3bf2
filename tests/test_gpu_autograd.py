"""F as a torch.autograd.Function whose backward is the hand-written adjoint sweep."""
import numpy as np
import pytest

import fixtures as F

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_3615_amd as M
    from paper_1101_3615_amd.autograd import born
    return M, born


def test_gradcheck_fp64():
    """torch.autograd.gradcheck of born() in FP64 on a small grid."""
    M, born = _gpu()
    w = F.tiny(n=12, nb=4, nt=40, ns=2, nr=6, dtype="f64", kind="smooth_random")
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(F.medium(w)))
    dm = torch.from_numpy(F.normal_field(w.model_shape, 3).astype(np.float64)).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: born(x, P), (dm,), eps=1e-3, atol=1e-7, rtol=1e-6,
                                    fast_mode=True)


def _c3_slice(snap, nshots=8):
    w = F.c3()
    sel = np.linspace(0, w.ns - 1, nshots).round().astype(int)
    return w.with_(src=w.src[sel], snap=snap)


@pytest.mark.parametrize("snap,tol", [("ckpt_f32", 1e-3), ("ckpt_bf16", 1e-2)])
def test_c3_slice_dot_product_and_finite_differences(snap, tol):
    """1024 x 512, 4000 steps, snapshots every 4 steps (8 of the 128 shots):
    dot-product test and central differences of L = 1/2 ||F dm - d_obs||^2 along
    32 seeded wavepacket directions (L is quadratic, so the central difference is
    exact up to rounding); tolerance FP32 checkpoints 1e-3, BF16 checkpoints 1e-2, on the
    relative L2 error of the 32 directional derivatives taken together and on each
    direction's own relative error (measured worst 3.1e-5 and 5.2e-3)."""
    M, born = _gpu()
    w = _c3_slice(snap)
    c = F.medium(w)
    P = M.Problem.from_spec(w)
    P.set_background(torch.from_numpy(c).cuda())
    refl = torch.from_numpy(F.reflectivity(w, c)).cuda()
    with torch.no_grad():
        d_obs = P.apply_F(refl).clone()
    dm0 = torch.from_numpy(F.wavepackets(w, c, 7, 64) * float(refl.abs().max())).cuda()
    x = dm0.clone().requires_grad_(True)
    r = born(x, P) - d_obs
    loss = 0.5 * (r.double() ** 2).sum()
    loss.backward()
    grad = x.grad.double()

    # dot-product test <F m, d> = <m, F* d> with band-limited vectors: m a wavepacket
    # sum, d the Born data of another one (with BF16 checkpoints F* is approximate,
    # and white-noise vectors would weigh the grid-scale part the rounding perturbs)
    m = torch.from_numpy(F.wavepackets(w, c, 8, 64)).cuda()
    dd = P.apply_F(torch.from_numpy(F.wavepackets(w, c, 9, 64)).cuda()).clone()
    lhs = float((P.apply_F(m).double() * dd.double()).sum())
    rhs = float((m.double() * P.apply_Fadj(dd).double()).sum())
    dot_err = abs(lhs - rhs) / abs(lhs)

    def L(v):
        with torch.no_grad():
            rr = (P.apply_F(v).double() - d_obs.double())
            return 0.5 * float((rr ** 2).sum())

    fds, ans = [], []
    for i in range(32):
        v = torch.from_numpy(F.wavepackets(w, c, 100 + i, 64)).cuda() * float(refl.abs().max())
        eps = 1.0
        fds.append((L(dm0 + eps * v) - L(dm0 - eps * v)) / (2 * eps))
        ans.append(float((grad * v.double()).sum()))
    fds, ans = np.array(fds), np.array(ans)
    errs = np.abs(fds - ans) / np.maximum(np.abs(fds), 1e-300)
    err_all = float(np.linalg.norm(fds - ans) / np.linalg.norm(fds))
    print(f"{snap}: dot-product rel err {dot_err:.3e}; FD vs backward over 32 directions: "
          f"relative L2 {err_all:.3e}, per direction median {np.median(errs):.3e}, max {errs.max():.3e}")
    assert dot_err <= tol
    assert err_all <= tol
    assert errs.max() <= tol
