"""Planted mistakes: copies of the oracle source with one plausible error
each (compiled on the CPU into a temporary directory) must fail at least one
of the pins that the real oracle passes.  This shows the pins can see a
dropped term, a wrong sign or index, a wrong offset direction or a swapped
operand anywhere in the oracle."""
import ctypes
import os

import numpy as np
import pytest

import oracle
from oracle import compile as obuild
from oracle import dense
from paper_1510_05218_amd import inputs

MUTATIONS = {
    # curl sign of H_yz flipped
    "sign_Hyz": ("/* H_yz */ {10, 11, 0, +1, -1},", "/* H_yz */ {10, 11, 0, -1, -1},"),
    # E_zx difference along x instead of y
    "axis_Ezx": ("/* E_zx */ { 0,  1, 1, -1, -1},", "/* E_zx */ { 0,  1, 0, -1, -1},"),
    # H_zx driven by the wrong split part (E_xy twice)
    "part_Hzx": ("/* H_zx */ { 6,  7, 1, +1, -1},", "/* H_zx */ { 6,  6, 1, +1, -1},"),
    # E uses a backward difference like H (offset direction of Fig. 3)
    "dir_E": ("const int dir = is_h ? -1 : +1;", "const int dir = -1;"),
    # the source term is dropped
    "no_src": ("const double *srcq = cm->src >= 0 ? coef[24 + cm->src] : NULL;",
               "const double *srcq = NULL;"),
    # phase factor of the H coefficient conjugated
    "phase_H": ("*t = conj(ph2) / d;", "*t = ph2 / d;"),
    # e^{-iwt/2} dropped from c_E
    "cE_phase": ("*c = (tau / (eps * h)) * conj(ph2) / d;", "*c = (tau / (eps * h)) / d;"),
    # real and imaginary parts of c swapped in the complex product c D
    "swap_c": ("double cd_r = cr * dr - ci * di, cd_i = cr * di + ci * dr;",
               "double cd_r = ci * dr - cr * di, cd_i = ci * di + cr * dr;"),
    # PML conductivity of H applied to the wrong components
    "pml_axis": ("double sst = (cq->axis == 2) ? sig_h[k] : 0.0;",
                 "double sst = (cq->axis == 1) ? sig_h[k] : 0.0;"),
    # E loss term dropped
    "no_loss": ("double sig_mat = omega * epp;", "double sig_mat = 0.0 * epp;"),
    # periodic wrap replaced by a wrong modulus
    "wrap": ("i = (i + g->nx) % g->nx;", "i = (i + g->nx - 1) % g->nx;"),
}


def _pins_pass():
    """The fixed-point identity on a random problem with every source array,
    both boundary types and a back-iteration cell."""
    for seed, bcx, bcy in ((31, 0, 0), (32, 1, 1)):
        pb = inputs.random_problem(5, 4, 8, seed=seed, bcx=bcx, bcy=bcy)
        pb.eps[2, 1, 1] = -2.0 + 0.5j
        coef = oracle.coeffs(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega, pb.tau)
        xs = dense.fixed_point(pb.eps, pb.sig_e, pb.sig_h, pb.sources, pb.omega,
                               pb.tau, bcx=bcx, bcy=bcy)
        y = oracle.phi(coef, xs, bcx, bcy)
        if np.linalg.norm(y - xs) > 1e-13 * np.linalg.norm(xs):
            return False
    return True


def test_real_oracle_passes(oracle_lib):
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(oracle_lib, tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"oracle_{name}.c"
    path.write_text(src.replace(old, new))
    so = obuild.compile_source(str(path), str(tmp_path / f"lib_{name}.so"))
    saved = oracle._lib
    oracle._lib = oracle._configure(ctypes.CDLL(os.path.abspath(so)))
    try:
        assert not _pins_pass(), f"planted mistake {name} not detected"
    finally:
        oracle._lib = saved
