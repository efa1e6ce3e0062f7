"""The oracle's design-loop gradient (blend, PDE filter, adjoint, filter
transpose) against central differences of its own objective and constraint."""
import numpy as np

from oracle import topopt as otop
from oracle.filter import Filter
from paper_1508_04596_amd import inputs


def test_design_gradient_matches_central_differences():
    p = inputs.cavity_problem(20, 1.0e3, s0=10.0)
    design = p.design
    rng = np.random.default_rng(4)
    rho = np.where(design, rng.uniform(0.3, 1.0, p.n_el), 0.0)
    gfix = p.gamma.copy()
    filt = Filter(p.nx, p.ny, p.nz, p.h, 2.5 * p.h)
    f, g, df, dg, _ = otop.evaluate(p, filt, rho, design, gfix, vf=0.05)
    d = np.where(design, rng.standard_normal(p.n_el), 0.0)
    eps = 1e-5
    fp, gp, _, _, _ = otop.evaluate(p, filt, rho + eps * d, design, gfix, vf=0.05, grads=False)
    fm, gm, _, _, _ = otop.evaluate(p, filt, rho - eps * d, design, gfix, vf=0.05, grads=False)
    fd_f, fd_g = (fp - fm) / (2 * eps), (gp - gm) / (2 * eps)
    assert abs(df @ d - fd_f) <= 1e-6 * abs(fd_f)
    assert abs(dg @ d - fd_g) <= 1e-8 * abs(fd_g)
    assert np.all(df[~design] == 0.0) and np.all(dg[~design] == 0.0)
