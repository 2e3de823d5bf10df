"""GPU: checkpoint and resume (mdx_state_size / mdx_save_state /
mdx_load_state). A run split by a save into one context and a load into a
fresh one must repeat the uninterrupted run bit for bit: the rebuild cadence,
the pruned list, the image counters, the Langevin step counter and the Kahan
terms all live in the saved state."""
import numpy as np
import pytest

import synth
from helpers import announce, gpu_context

pytestmark = pytest.mark.gpu


def _run(s, chunks, langevin, options, save_after=None):
    """Integrates s for sum(chunks) steps. With save_after = k, the state is
    saved after the first k chunks and the remaining chunks run in a fresh
    context loaded from it. Returns pos, vel, images."""
    import torch
    import paper_2503_20541_amd as mdx
    dev = torch.device("cuda:0")
    with gpu_context(s, options=options) as (m, ctx, t):
        m.build_neighbors(ctx, t["pos"])
        m.compute_nonbonded(ctx, t["pos"], t["force"])
        if s.pme_grid[0]:
            m.compute_pme(ctx, t["pos"], t["force"])
        if langevin:
            m.set_langevin(ctx, *langevin)
        head = chunks if save_after is None else chunks[:save_after]
        for k in head:
            m.integrate_step(ctx, t["pos"], t["vel"], t["force"], k, float(s.dt))
        if save_after is None:
            img = torch.zeros((3, s.n_atoms), dtype=torch.int32, device=dev)
            m.get_images(ctx, img)
            torch.cuda.synchronize()
            assert m.get_status(ctx) == 0
            return t["pos"].cpu().numpy(), t["vel"].cpu().numpy(), img.cpu().numpy()
        nbytes = m.state_size(ctx)
        state = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        m.save_state(ctx, state)
        saved = {k: t[k].clone() for k in ("pos", "vel", "force")}
        torch.cuda.synchronize()
        assert m.get_status(ctx) == 0
    # the first context is gone; a fresh one continues from the state
    with gpu_context(s, options=options) as (m, ctx, t):
        for k in ("pos", "vel", "force"):
            t[k].copy_(saved[k])
        if langevin:
            m.set_langevin(ctx, *langevin)
        m.load_state(ctx, state)
        for k in chunks[save_after:]:
            m.integrate_step(ctx, t["pos"], t["vel"], t["force"], k, float(s.dt))
        img = torch.zeros((3, s.n_atoms), dtype=torch.int32, device=dev)
        m.get_images(ctx, img)
        torch.cuda.synchronize()
        assert m.get_status(ctx) == 0
        assert m.get_info(ctx).steps_taken == sum(chunks)
        return t["pos"].cpu().numpy(), t["vel"].cpu().numpy(), img.cpu().numpy()


@pytest.mark.parametrize("name,langevin,options", [
    ("water375", (0.596, 0.1, 20541), 0),          # PME water, Langevin 300 K
    ("water9k", None, 0),                           # PME water, velocity Verlet
    ("lj1k", None, 0x4),                            # MDX_OPT_KAHAN_VV
    ("water9k", None, 0x1),                         # MDX_OPT_HALF_LIST
])
def test_resume_from_saved_state_is_bitwise(name, langevin, options):
    s = synth.config_system(name)
    chunks = [7, 6, 10]           # the save lands between rebuilds (cadence 10)
    announce(f"state {name} langevin={langevin is not None} options={options}")
    ref = _run(s, chunks, langevin, options)
    res = _run(s, chunks, langevin, options, save_after=2)
    for a, b in zip(ref, res):
        assert np.array_equal(a, b)


def test_state_errors():
    import torch
    s = synth.config_system("water375")
    announce("state errors")
    with gpu_context(s) as (m, ctx, t):
        m.build_neighbors(ctx, t["pos"])
        n = m.state_size(ctx)
        assert n > 0 and n % 256 == 0
        buf = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
        with pytest.raises(m.MdxError) as e:
            m.save_state(ctx, buf, capacity=n - 1)
        assert e.value.code == m.MDX_E_CAPACITY
        with pytest.raises(m.MdxError) as e:          # zeros: not a state
            m.load_state(ctx, buf)
        assert e.value.code == m.MDX_E_INVALID
        m.save_state(ctx, buf)
        with pytest.raises(m.MdxError) as e:          # shorter than the state
            m.load_state(ctx, buf, size=n - 256)
        assert e.value.code == m.MDX_E_INVALID
        m.load_state(ctx, buf)                        # its own state loads back
        torch.cuda.synchronize()
    other = synth.config_system("lj1k")
    with gpu_context(other) as (m, ctx, t):
        with pytest.raises(m.MdxError) as e:          # another system
            m.load_state(ctx, buf)
        assert e.value.code == m.MDX_E_INVALID
