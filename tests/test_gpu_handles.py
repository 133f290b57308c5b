"""Handle lifetimes through the C ABI: every handle may be destroyed after
the context (and grid) it was made with, in any order, and leaves no device
error behind for the next context's work (the destroy calls free on the
device recorded in the handle instead of reading the context)."""
import numpy as np
import pytest

from amr_inputs import random_amr
from amr_inputs.mlp_init import glorot_init

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1509_07370_amd import binding as B  # noqa: E402


def _handles():
    g = random_amr(5, nbase=2, max_level=1, p_refine=0.3)
    ctx = B.bh_ctx_create(0)
    grid = B.bh_grid_create_from(ctx, g)
    rho = torch.tensor(g.rho, device="cuda")
    m = B.bh_build_moments(ctx, grid, rho, None)
    lists = B.bh_walk(ctx, grid, m, 0.5)
    table = B.bh_ewald_create(ctx, g.box_size, 9)
    net = B.bh_mlp_create(ctx, glorot_init(3).astype(np.float32), np.zeros(12, np.float32),
                          np.ones(12, np.float32))
    batch = B.bh_batch_create(ctx, [grid])
    torch.cuda.synchronize()
    return g, rho, ctx, grid, dict(moments=m, lists=lists, table=table, net=net, batch=batch)


@pytest.mark.parametrize("order", [("batch", "net", "table", "lists", "moments"),
                                   ("moments", "lists", "table", "net", "batch")])
def test_handles_outlive_their_context(order):
    g, rho, ctx, grid, h = _handles()
    B.bh_ctx_destroy(ctx)
    B.bh_grid_destroy(grid)
    destroy = dict(moments=B.bh_moments_destroy, lists=B.bh_lists_destroy, table=B.bh_ewald_destroy,
                   net=B.bh_mlp_destroy, batch=B.bh_batch_destroy)
    for name in order:
        destroy[name](h[name])
    # a fresh context works, with no error left over from the destroy calls
    ctx2 = B.bh_ctx_create(0)
    grid2 = B.bh_grid_create_from(ctx2, g)
    m2 = B.bh_build_moments(ctx2, grid2, rho, None)
    phi = torch.empty_like(rho)
    B.bh_walk_potential(ctx2, grid2, m2, 0.5, None, B.BH_FP64, 1.0, phi, None)
    B.bh_moments_check(ctx2, m2)
    assert torch.isfinite(phi).all()
    B.bh_moments_destroy(m2)
    B.bh_grid_destroy(grid2)
    B.bh_ctx_destroy(ctx2)
