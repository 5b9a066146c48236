"""Symmetric path: the interior and interface operators stored packed against the same
preconditioner stored whole.

Packed, the symmetric blocks K_II^-1 and D S~ D are stored once, as lower column panels (every
stored tile read once per application for both its product and its transposed product), and the
interior correction is solved as z_I = K_II^-1 (r_I - K_IG z_G) with K_IG on its sparse pattern,
so that phase A multiplies by G alone; whole, phase A multiplies by [K_II^-1; G] and phase H
subtracts H z_G with H = G^T stored (paper §3.2 block factorisation, either form).

packed_sym = 2 forces the packed layout (1, the default, takes it when it saves 10 % of the
operator bytes, i.e. for blocks of several panels). The two are different roundings of the same
operator: one application agrees within the apply bounds of the oracle parity tests (FP64:
max(1e-12, 100 x the oracle's own noise floor); mixed: 1e-5), GMRES takes the same number of
iterations (+-1; mixed +-2) and both solutions meet the tolerance. Cases span one and many panels
per block (local blocks of 81 to 4.4k rows), ragged panel tails, two and three levels, and every
right-hand-side width. The agreement with the oracle is checked by the parity tests, which run
the packed layout (the default)."""
import numpy as np
import pytest

from paper_2208_06191_amd import mbddc
from tests.conftest import apply_noise_floor, problem

pytestmark = pytest.mark.gpu


def solver(P, precision, packed, levels=2, primal=None):
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)],
                           mbddc.default_options(precision=precision, primal=primal or P.primal, symmetric_hint=1,
                                                 levels=levels, packed_sym=packed))
    s.mbddc_set_tangent(P.Ke)
    s.mbddc_factor()
    return s


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("precision", [mbddc.MBDDC_FP64, mbddc.MBDDC_MIXED])
@pytest.mark.parametrize("name,levels", [("small_ve", 2), ("ragged", 2), ("vent", 2), ("large_q1", 2),
                                         ("vent_parts6k", 2), ("l3_nh", 3), ("vent", 3)])
def test_packed_equals_full_layout(name, levels, precision):
    P = problem(name)
    sp, sf = solver(P, precision, 2, levels), solver(P, precision, 0, levels)   # packed forced / whole
    if name in ("large_q1", "vent_parts6k"):   # blocks of many panels: less memory, and chosen by default
        assert sp.mbddc_footprint(1) < sf.mbddc_footprint(1)
        sd = solver(P, precision, 1, levels)
        assert sd.mbddc_footprint(1) == sp.mbddc_footprint(1)
        sd.close()
    if precision == mbddc.MBDDC_FP64:
        bound = max(1e-12, 100.0 * apply_noise_floor(name, P.primal, levels=levels))
    else:
        bound = 1e-5
    rng = np.random.default_rng(2)
    for nrhs in (1, 2, 3, 8):
        r = rng.standard_normal((nrhs, P.n_dofs))
        r[:, P.dirichlet] = 0.0
        zp, zf = sp.mbddc_apply(r), sf.mbddc_apply(r)
        e = max(rel(zp[k], zf[k]) for k in range(nrhs))
        assert e <= bound, (nrhs, e, bound)
    xp, ip = sp.mbddc_solve(P.rhs)
    xf, if_ = sf.mbddc_solve(P.rhs)
    print(f"{name} levels {levels} prec {precision}: apply agreement {e:.1e} (bound {bound:.1e}), its "
          f"{ip.iterations} / {if_.iterations}, footprint {sp.mbddc_footprint(1) / 1e6:.1f} / "
          f"{sf.mbddc_footprint(1) / 1e6:.1f} MB")
    assert abs(ip.iterations - if_.iterations) <= (1 if precision == mbddc.MBDDC_FP64 else 2)
    assert ip.rel_res_true <= 1e-8 and if_.rel_res_true <= 1e-8
    sp.close()
    sf.close()
