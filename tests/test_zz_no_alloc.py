"""The allocation-free J v entry point (fe_jvp_noalloc) against fe_jvp.

For callers that cannot allocate device memory.  Same kernels as fe_jvp, so the
products must be bitwise equal to fe_jvp's on a problem with the same grid,
parameters and mask.  Two calls in a row share the library's static scratch
array, the second with a smaller grid; sizes beyond the scratch are refused
before anything is launched, and so is every call that gives a short tensor."""
import numpy as np
import pytest

from paper_1508_04596_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_04596_amd import fe as fe_mod
    fe_mod.lib()
    return fe_mod


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def _both(fe, p, mask_kind, prec, seed):
    m = {"solve": p.mask_solve, "walls": p.mask_walls, None: None}[mask_kind]
    dt = torch.float64 if prec == "fp64" else torch.float32
    x = dev(inputs.random_state(p, seed, mask=m if m is not None else p.mask_walls), dt)
    v = dev(np.random.default_rng(seed + 1).standard_normal(p.n_dof), dt)
    g, s = dev(p.gamma), dev(p.s)
    ph = fe.make_phys(p.Pr, p.Gr, p.Ck, p.qf, p.alpha_max, p.q_alpha, p.eg)
    md = None if m is None else dev(m, torch.uint8)
    out = fe.fe_jvp_noalloc(p.nx, p.ny, p.nz, p.h, ph, md, x, g, s, v)
    prob = fe.Problem(p.nx, p.ny, p.nz, p.h, ph, md)
    ref = fe.fe_jvp(prob, x, g, s, v)
    torch.cuda.synchronize()
    prob.close()
    return out, ref


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_jvp_equals_fe_jvp_twice_second_smaller(fe, prec):
    big = inputs.scaled_config(40, 24, 19, 1e4, seed=61)      # 5 x 3 x 5 tiles, ragged
    small = inputs.scaled_config(13, 7, 9, 3e3, seed=62)      # ragged, fewer tiles
    for p, mk in ((big, "solve"), (small, "walls")):
        print(f"[noalloc] {prec} {p.nx}x{p.ny}x{p.nz} mask={mk}", flush=True)
        out, ref = _both(fe, p, mk, prec, seed=7)
        assert torch.equal(out, ref), f"{p.nx}x{p.ny}x{p.nz}: differs from fe_jvp"


def test_noalloc_jvp_without_mask_and_at_the_largest_accepted_size(fe):
    # no mask at all
    p = inputs.scaled_config(9, 8, 5, 2e3, seed=63)
    out, ref = _both(fe, p, None, "fp64", seed=3)
    assert torch.equal(out, ref)
    # 96^3 in FP64 needs 56.8 MB of the 64 MiB scratch
    n = 96
    need = fe.fe_jvp_noalloc_scratch_bytes(n, n, n)
    assert need <= fe.FE_NOALLOC_SCRATCH_BYTES
    p = inputs.scaled_config(n, n, n, 1e5, seed=64)
    out, ref = _both(fe, p, "solve", "fp64", seed=5)
    assert torch.equal(out, ref)


def test_noalloc_refuses_grids_beyond_the_scratch(fe):
    n = 128  # 16 x 16 x 32 tiles: 133 MB in FP64
    assert fe.fe_jvp_noalloc_scratch_bytes(n, n, n) > fe.FE_NOALLOC_SCRATCH_BYTES
    ph = fe.make_phys()
    nd, ne = 5 * (n + 1) ** 3, n ** 3
    z = torch.zeros(nd, dtype=torch.float64, device="cuda")
    ge = torch.zeros(ne, dtype=torch.float64, device="cuda")
    with pytest.raises(fe.FeError) as ei:
        fe.fe_jvp_noalloc(n, n, n, 1.0 / n, ph, None, z, ge, ge, z, out=z.clone())
    assert ei.value.code == fe.FE_EINVAL and "scratch" in str(ei.value)
    with pytest.raises(ValueError):
        fe.fe_jvp_noalloc(4, 4, 4, 0.25, ph, None, z[:10], ge[:64], ge[:64], z[:10])
