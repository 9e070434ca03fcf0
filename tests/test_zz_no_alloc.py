"""bdem_create_in_scratch (the allocation-free variant of bdem_create, whose
workspace is the library's static device array) against bdem_create: the
same steps from the same state give the same bits, on two handles created one
after the other in the array, the second for a smaller problem.  Also: a
second live handle in the array and a problem larger than the array are
refused with their documented codes."""
import numpy as np
import pytest

from paper_2308_10459_amd import scenes as S
from tests.gpu_helpers import log, make_sim

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_10459_amd import bdem
    return bdem


def _run(B, scene, mixed, in_scratch, steps):
    sim = make_sim(scene, mixed=mixed, in_scratch=in_scratch)
    rcs = []
    for _ in range(steps):
        st = sim.step(scene.dt)
        rcs.append((st["rc"], st["newton_iters"], st["cg_iters"], st["bonds_broken"]))
    out = sim.get_state()
    sim.close()
    return out, rcs


@pytest.mark.parametrize("mixed", [False, True])
def test_create_in_scratch_matches_create(B, mixed):
    # two calls in a row in the same array, the second with a smaller problem
    scenes = [S.make_plate_drop(nx=24, ny=20, nl=2, sigma_c=3e5, tau_c=3e5),
              S.make_block(nx=6, ny=5, nz=4)]
    assert scenes[1].n < scenes[0].n
    for sc in scenes:
        ref, rref = _run(B, sc, mixed, False, 3)
        got, rgot = _run(B, sc, mixed, True, 3)
        log(f"[in scratch] {sc.name} mixed={mixed}: steps {rgot} (bdem_create: {rref})")
        assert rgot == rref
        for k in ("pos", "quat", "vel", "qvel", "alive"):
            np.testing.assert_array_equal(got[k], ref[k])


def test_create_in_scratch_refusals(B):
    sc = S.make_block(nx=4, ny=4, nz=4)
    a = make_sim(sc, in_scratch=True)
    with pytest.raises(B.BdemError) as e:
        make_sim(sc, in_scratch=True)
    assert e.value.code == B.BDEM_E_STATE
    a.close()
    # released: a new handle may take the array
    b = make_sim(sc, in_scratch=True)
    b.step(sc.dt)
    b.close()
    # a problem larger than the array
    big = S.make_plate_drop()
    assert B.bdem_workspace_bytes(big, B.scene_options(big)) > B.BDEM_SCRATCH_BYTES
    with pytest.raises(B.BdemError) as e:
        make_sim(big, in_scratch=True)
    assert e.value.code == B.BDEM_E_NOMEM
    assert "static scratch" in str(e.value)
    # the multigrid hierarchy would need its own allocation
    with pytest.raises(B.BdemError) as e:
        make_sim(sc, in_scratch=True, preconditioner=B.BDEM_PRECOND_AMG)
    assert e.value.code == B.BDEM_E_INVALID
    # the refusals left the array free
    c = make_sim(sc, in_scratch=True)
    c.close()
