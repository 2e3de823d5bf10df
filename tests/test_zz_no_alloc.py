"""GPU: mdx_compute_ewald_direct_noalloc (the direct reciprocal Ewald sum with
the library's fixed scratch array, no allocation) against
mdx_compute_ewald_direct on the same inputs, bit for bit, on two calls in a
row (the second with a smaller system and n_max), and against the oracle's
direct sum."""
import numpy as np
import pytest

import synth
from oracle import ewald, forcefield
from helpers import announce, gpu_context, rel_rms

pytestmark = pytest.mark.gpu


def _both(name, n_max):
    import torch
    s = synth.config_system(name)
    announce(f"direct Ewald no-alloc {name} n_max={n_max}")
    with gpu_context(s) as (mdx, ctx, t):
        out = {}
        for fn in ("noalloc", "alloc"):
            e = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
            f = torch.zeros_like(t["force"])
            if fn == "noalloc":
                mdx.compute_ewald_direct_noalloc(ctx, t["pos"], f, e, n_max)
            else:
                mdx.compute_ewald_direct(ctx, t["pos"], f, e, n_max)
            torch.cuda.synchronize()
            out[fn] = (f.cpu().numpy(), float(e.cpu()[0]))
    return s, out


@pytest.mark.parametrize("name,n_max", [("water9k", 10), ("water375", 6)])
def test_noalloc_matches_allocating_call(name, n_max):
    s, out = _both(name, n_max)
    (fa, ea), (fb, eb) = out["noalloc"], out["alloc"]
    assert np.array_equal(fa, fb)
    assert ea == eb
    a = forcefield.alpha(s)
    Eref, Fref = ewald.reciprocal_direct(s.pos.astype(np.float64), s.charge, s.box, a,
                                         s.coulomb_k, n_max)
    assert abs(ea - Eref) <= 1e-9 * abs(Eref), (ea, Eref)
    assert rel_rms(fa, Fref) < 1e-6


def test_noalloc_rejects_scratch_beyond_the_array():
    import torch
    s = synth.config_system("water9k")
    announce("direct Ewald no-alloc capacity")
    with gpu_context(s) as (mdx, ctx, t):
        need, limit = mdx.ewald_direct_noalloc_bytes(s.n_atoms, 40)
        assert need > limit == 32 << 20
        with pytest.raises(mdx.MdxError) as e:
            mdx.compute_ewald_direct_noalloc(ctx, t["pos"], t["force"], None, 40)
        assert e.value.code == mdx.MDX_E_CAPACITY
        torch.cuda.synchronize()
        assert not t["force"].any()      # nothing ran
