"""Pins of the oracle's operation count (the flop roofline's denominator).

Every expected number below is counted by hand from the formulas of the step
(Sec. 2.2: primitive variables, generalized-minmod PLM, Hancock half step,
HLLC, conservative update), each add/sub, mul, div and sqrt once, negation
free.  A counting scalar that missed an operation kind, a stage that gained
or lost a term, or a branch counted on the wrong path fails one of them.
"""

import json
import os

import numpy as np

import oracle
from oracle import count_flops

G53 = 5.0 / 3.0
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def ops(**kw):
    U, Wc, Wm, Wp, UL, UR, gamma = count_flops.stage_inputs()
    a = dict(U=U, Wc=Wc, Wm=Wm, Wp=Wp, UL=UL, UR=UR)
    a.update(kw)
    return oracle.count_ops(a["U"], a["Wc"], a["Wm"], a["Wp"], a["UL"], a["UR"], gamma, 1.5, 0.01)


def t(add, mul, div, sqrt):
    return {"add": add, "mul": mul, "div": div, "sqrt": sqrt}


def test_cons_to_prim_count():
    # u, v, w: 3 div; m.u = mx u + my v + mz w: 3 mul 2 add;
    # p = (g-1) (E - 0.5 m.u): 2 mul 1 add
    assert ops()["cons_to_prim"] == t(3, 5, 3, 0)


def test_hancock_count_all_limiters_active():
    # per (axis, variable), 15 of them: dm, dp (2 add); one sign -> dc = 0.5 (qp - qm)
    #   (1 add 1 mul), theta|dm|, theta|dp| (2 mul); faces q0 -+ 0.5 s (2 mul 2 add)
    #   -> 5 add 5 mul, 75 / 75 in all
    # per face state, 6 of them: cons (rho u, rho v, rho w: 3 mul; u^2+v^2+w^2:
    #   3 mul 2 add; p/(g-1) + 0.5 rho |v|^2: 1 div 2 mul 1 add) and flux
    #   (4 mul, +p on the normal momentum 1 add, (E+p) u_n 1 add 1 mul)
    #   -> 5 add 13 mul 1 div, 30 / 78 / 6 in all
    # per variable, 5 of them: sum of three flux differences 5 add, times
    #   dt/(2dx) 1 mul, added to 6 face states 6 add -> 55 add 5 mul
    assert ops()["hancock_cell"] == t(75 + 30 + 55, 75 + 78 + 5, 6, 0)


def test_hancock_count_no_limiter_active():
    # flat neighbourhood: every slope is zero after dm, dp (2 add) and the faces
    # still take q0 -+ 0.5 s (2 mul 2 add): 15 x (4 add, 2 mul)
    U, Wc, *_ = count_flops.stage_inputs()
    flat = np.tile(Wc, 3)
    assert ops(Wm=flat, Wp=flat)["hancock_cell"] == t(60 + 30 + 55, 30 + 78 + 5, 6, 0)


# HLLC, common part: u, v, w of both sides 6 div; p of each side
# (g-1)(E - 0.5 rho (u^2+v^2+w^2)) 6 mul 3 add -> 12 mul 6 add; c of each side
# sqrt(g p / rho) 1 mul 1 div 1 sqrt -> 2 mul 2 div 2 sqrt; Roe speeds: sqrt rho
# twice, 1/(sL+sR) 1 add 1 div, three averaged velocities 3 mul 1 add each,
# H of each side (E+p)/rho 1 add 1 div, averaged H 3 mul 1 add, c~ = sqrt((g-1)
# (H~ - 0.5 |u~|^2)) 5 mul 3 add 1 sqrt, S_L and S_R from two sums each 4 add
# -> 17 mul 14 add 3 div 3 sqrt; S* 8 add 6 mul 1 div; both physical fluxes
# 8 mul 4 add.
HLLC_COMMON = (6 + 14 + 8 + 4, 12 + 2 + 17 + 6 + 8, 6 + 2 + 3 + 1, 5)


def test_hllc_count_star_branch():
    # star flux of one side: r = (S-u)/(S-S*) 2 add 1 div; U* (rho, rho S*, m_t1,
    # m_t2: 5 mul; energy: S-u, p/(S-u), rho S*, +, S*-u, x, E+, r x: 4 add 3 mul
    # 1 div); F + S (U* - U) per variable 2 add 1 mul -> 16 add 13 mul 2 div
    a, m, d, s = HLLC_COMMON
    assert ops()["hllc_flux"] == t(a + 16, m + 13, d + 2, s)


def test_hllc_count_supersonic_branch():
    # S_L >= 0: the left physical flux, already formed, nothing more
    UL = oracle.prim_to_cons(np.array([1.0, 5.0, 0.1, 0.0, 1.0]), G53)
    UR = oracle.prim_to_cons(np.array([0.8, 4.5, 0.0, 0.1, 0.9]), G53)
    a, m, d, s = HLLC_COMMON
    assert ops(UL=UL, UR=UR)["hllc_flux"] == t(a, m, d, s)


def test_update_count():
    # per variable: three flux differences summed 5 add, U - (dt/dx) acc 1 add 1 mul;
    # check of the new state p = (g-1)(E - 0.5 |m|^2 / rho): 3 mul 2 add, 0.5 x
    # 1 mul, / rho 1 div, E - 1 add, (g-1) x 1 mul
    assert ops()["update"] == t(30 + 3, 5 + 5, 1, 0)


def test_multiplicities_by_enumeration():
    # interior 16^3 plus 6 face layers of 16^2 state cells; their stencil adds a
    # second face layer (6 x 256) and the 12 edge lines of 16 cells
    assert len(count_flops.state_cells()) == 16 ** 3 + 6 * 256
    assert len(count_flops.reachable_cells()) == 16 ** 3 + 2 * 6 * 256 + 12 * 16
    assert count_flops.faces() == 3 * 17 * 256


def test_committed_flop_count_is_the_scripts():
    with open(os.path.join(ROOT, "oracle", "flops_per_cell.json")) as fh:
        stored = json.load(fh)
    rec = count_flops.count()
    assert stored["flops_per_cell_update"] == rec["flops_per_cell_update"]
    assert stored["ops_per_item"] == rec["ops_per_item"]
    # hand total: 11 x 7360 + 324 x 5632 + 125 x 13056 + 44 x 4096 per group
    assert rec["per_group"] == 11 * 7360 + 324 * 5632 + 125 * 13056 + 44 * 4096
