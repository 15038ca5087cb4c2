"""The allocation-free entry point (nb_compute_forces_noalloc) against the
allocating one (nb_sys_create + nb_sys_set_particles + nb_compute_forces), called
through the C ABI: two calls in a row on the library's one scratch array, the
second with a smaller system; forces, energies and virial bitwise equal, and
within the 1e-5 rel-RMS force tolerance of the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1506_00716_amd import inputs

pytestmark = pytest.mark.gpu


def allocating(nbmod, ctx, s, x):
    import torch
    g = nbmod.System(ctx, s)
    f = torch.zeros((s.n, 3), dtype=torch.float32, device=ctx.device)
    g.build_pairlist(x)
    e, w = g.compute_forces(x, f)
    g.close()
    return f.cpu().numpy(), e, w


def test_noalloc_equals_allocating_entry_point(nbmod, gpu_ctx):
    import torch
    big = inputs.small_rf()  # 2,700 atoms, reaction field
    lb = inputs.Model(r_cut=0.9, r_list=1.0, coulomb="ewald", ewald_beta=3.12, lj="lb")
    small = inputs.tiny_random_system(777, [3.1, 3.3, 3.2], 31, lb, min_dist=0.17)  # Ewald + LB
    for s in (big, small):
        print(f"[noalloc] N={s.n} coul={s.model.coulomb} lj={s.model.lj}", flush=True)
        x = torch.tensor(s.x, dtype=torch.float64, device=gpu_ctx.device)
        f = torch.full((s.n, 3), float("nan"), dtype=torch.float32, device=gpu_ctx.device)
        e, w = nbmod.compute_forces_noalloc(gpu_ctx, s, x, f)
        fn = f.cpu().numpy()
        fa, ea, wa = allocating(nbmod, gpu_ctx, s, x)
        assert np.array_equal(fn, fa)
        assert np.array_equal(e, ea) and np.array_equal(w, wa)
        fr, er, _ = oracle.forces(s)
        err = float(np.sqrt(((fn - fr) ** 2).sum() / (fr ** 2).sum()))
        print("rel-RMS vs oracle", err, flush=True)
        assert err <= 1e-5


def test_noalloc_rejects_a_system_beyond_the_array(nbmod, gpu_ctx):
    import torch
    big = inputs.lattice_system(200_000, 12.6, 3, inputs.MODEL_EWALD)
    pb = nbmod.make_params(big.n, big.box, big.model)
    assert nbmod.arena_bytes(pb) > nbmod.NOALLOC_MAX_BYTES
    x = torch.tensor(big.x, dtype=torch.float64, device=gpu_ctx.device)
    f = torch.zeros((big.n, 3), dtype=torch.float32, device=gpu_ctx.device)
    with pytest.raises(nbmod.NbError) as exc:
        nbmod.compute_forces_noalloc(gpu_ctx, big, x, f)
    assert exc.value.code == nbmod.NB_ERR_CAPACITY
