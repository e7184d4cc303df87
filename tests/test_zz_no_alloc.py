"""pond_step_noalloc, the entry point that allocates no device memory, against pond_step:
the same kernels on caller-owned state buffers with a static scratch array, so the
states after the same steps must be bitwise equal (two calls in a row, the second on a
smaller lattice, which must also be unaffected by what the first left in the scratch).
"""
import ctypes

import numpy as np
import pytest

from paper_2002_09217_amd import pond, workloads as W
from tests.common import pond_config

pytestmark = pytest.mark.gpu


def state_bytes(cfg):
    q = 9 if cfg.dim == 2 else 3
    pops = 2 * q * 8 if cfg.precision == pond.FP64 else 2 * q * 4 + 16
    return cfg.N * (pops + 5 * 8)


def run_both(torch, case, precision, steps, tile):
    """Step one state with pond_step and with pond_step_noalloc; return both states."""
    print(f"no-alloc case {case.name} n={case.n} precision={precision} tile={tile} steps={steps}", flush=True)
    cfg = pond_config(case, precision, stream=torch.cuda.current_stream().cuda_stream, tile=tile)
    cfg.two_kernel = 1   # the form with stored populations, which pond_step_noalloc runs
    lat = pond.Lattice(cfg)
    try:
        lat.init_fields(case.rho, case.u, case.T)
        ck0 = lat.save()
        lat.step(steps)
        ck1 = lat.save()
    finally:
        lat.close()
    nb = state_bytes(cfg)
    head = len(ck0) - nb
    bufs = [torch.from_numpy(np.frombuffer(ck0[head:], dtype=np.uint8).copy()).cuda(),
            torch.full((nb,), 0xAB, dtype=torch.uint8, device="cuda")]
    torch.cuda.synchronize()
    rc, cur, done = pond.step_noalloc(cfg, bufs[0].data_ptr(), bufs[1].data_ptr(), 0, steps)
    assert rc == pond.POND_OK, pond.STATUS.get(rc, rc)
    assert done == steps and cur == steps % 2
    got = bufs[cur].cpu().numpy().tobytes()
    ref = ck1[head:]
    if cfg.dim == 1:
        # 1D lattices neither read nor write the side planes u_y and F_y: leave them out
        pops = nb - 5 * 8 * cfg.N
        plane = lambda b, k: b[pops + k * 8 * cfg.N: pops + (k + 1) * 8 * cfg.N]
        keep = lambda b: b[:pops] + b"".join(plane(b, k) for k in (0, 2, 3))
        got, ref = keep(got), keep(ref)
    return got, ref


@pytest.mark.parametrize("precision", [pond.FP64, pond.FP32_STORE])
def test_noalloc_matches_pond_step_twice(precision):
    torch = pytest.importorskip("torch")
    assert torch.cuda.is_available()
    big = W.static_droplet(n=96, radius=20.0)
    got, ref = run_both(torch, big, precision, 7, tile=5)
    assert got == ref
    # a second call right after, on a smaller, ragged lattice with another tile shape
    small = W.perturbed(nx=40, ny=36, seed=3)
    got, ref = run_both(torch, small, precision, 4, tile=2)
    assert got == ref


def test_noalloc_one_dimensional():
    torch = pytest.importorskip("torch")
    got, ref = run_both(torch, W.shock_tube(n=300), pond.FP64, 5, tile=0)
    assert got == ref


def test_noalloc_rejects_a_lattice_beyond_the_scratch():
    torch = pytest.importorskip("torch")
    # 700 x 700 nodes need 4096 + 18 * 8 * 490000 bytes > 64 MiB
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    cfg = pond.Config(dim=2, n=(700, 700), tile=0, two_kernel=1)
    rc, cur, done = pond.step_noalloc(cfg, buf.data_ptr(), buf.data_ptr(), 0, 1)  # rejected before any launch
    assert rc == -8 and cur == 0 and done == 0
    cfg = pond.Config(dim=2, n=(16, 16), tile=0, two_kernel=1)
    assert pond.step_noalloc(cfg, 0, buf.data_ptr(), 0, 1)[0] == -1   # NULL buffer
    assert pond.step_noalloc(cfg, buf.data_ptr(), buf.data_ptr(), 2, 1)[0] == -1   # cur not 0 or 1
