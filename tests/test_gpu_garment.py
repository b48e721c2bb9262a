"""GPU parity of the garment (Baraff-Witkin membrane, Sec. IV-D) dropped onto a fixed
cone, the paper's coupling example: 121 vertices, 200 triangles, dt = 0.005 s.

  * every Newton iterate of the oracle's first 8 steps (free fall, first contact with
    the apex, draping): candidate sets bit-identical, energy terms within 1e-9, per-term
    gradients (the elastic term carries the garment) and H v within 1e-9;
  * the library's own trajectory over the same steps: the same Newton iteration counts,
    positions within 1e-9 m of the oracle's, no intersection at the end (exact check).
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import exact, ref
from test_gpu_parity import check_grad_terms, check_hv, check_terms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STEPS = 8


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def zema():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_05945_amd import zema as z
    return z


def grad_floor(sc, y):
    """Rounding floor of the membrane gradient: a triangle's columns w = sum_a c_a x_a
    (|c_a| ~ 1/edge) carry an absolute error of a few eps sum |c_a| |x_a|, so near rest
    |w| - 1 is rounding and the gradient h^2 A k_s (|w| - 1) c_a of ~6 triangles per
    vertex is bounded by 64 eps h^2 k_s max|x| (A |c_a| ~ edge, sum |c_a| |x_a| ~
    3 max|x| / edge)."""
    return 64 * np.finfo(float).eps * sc.params.dt ** 2 * sc.softs[0].E * np.abs(y).max()


def garment():
    sc = sg.garment_on_cone(gap=2e-3, steps=STEPS)
    sc.params.dt = 0.005
    return sc


@pytest.fixture(scope="module")
def iterates():
    sc = garment()
    R = ref.RefScene(sc)
    R.record(True)
    st = R.step(STEPS)
    return sc, R.records(), st


def test_garment_iterates_follow_oracle(zema, iterates):
    sc, recs, _ = iterates
    R = ref.RefScene(sc)
    G = zema.Scene(sc)
    # rounding floor of the energy terms: 64 eps times the membrane energy of unit
    # strain over the sheet, h^2 k_s A (k_s = E in N/m, A = 0.3^2 m^2)
    floor = 64 * np.finfo(float).eps * sc.params.dt ** 2 * sc.softs[0].E * 0.3 ** 2
    for i, rc in enumerate(recs):
        for S in (R, G):
            S.set_state(rc["y_t"], rc["ydot_t"], rc["kappa_lag"], rc["step"])
            S.set_kappa(rc["kappa"])
        y = rc["y_k"]
        xs = R.surface_positions(y)
        pr, er = R.candidates(xs, None)
        pg, eg = G.contact_candidates(xs, None)
        assert np.array_equal(pg.cpu().numpy(), pr) and np.array_equal(eg.cpu().numpy(), er), f"iterate {i}"
        tr, _ = R.ip_assemble(y, hess=False)
        tg, _ = G.ip_assemble(y, hess=False)
        check_terms(tg, tr, f"iterate {i}", floor)
        w = check_grad_terms(G, R, y, f"iterate {i}", rc["y_t"], term_floor={1: grad_floor(sc, y)})
        wh = check_hv(G, R, y, i, f"iterate {i}", masks=(0, 1 << 1, 1 << 4, 1 << 5))
        log(f"iterate {i} (step {rc['step']}): {len(pr)} PT + {len(er)} EE candidates, elastic {tr[1]:.3e}, "
            f"barrier {tr[4]:.3e}; worst gradient {w:.1e}, H v {wh:.1e}")
    log(f"{len(recs)} iterates")


def test_garment_trajectory_follows_oracle(zema, iterates):
    sc, _, so = iterates
    R = ref.RefScene(sc)
    G = zema.Scene(sc)
    sg_ = G.step(STEPS)
    R.step(STEPS)
    dy = np.abs(G.get_state()[0].cpu().numpy() - R.get_state()[0]).max()
    log(f"Newton gpu {[x['newton_iters'] for x in sg_]} oracle {[x['newton_iters'] for x in so]}, |y - y_oracle| {dy:.2e}")
    assert all(x["status"] == 0 for x in sg_)
    assert [x["newton_iters"] for x in sg_] == [x["newton_iters"] for x in so]
    assert dy <= 1e-9
    tris, edges, vb = (t.cpu().numpy() for t in G.surface_view()[:3])
    y = G.get_state()[0].cpu().numpy()
    assert exact.count_intersections(R.surface_positions(y), tris, edges, vb) == 0
