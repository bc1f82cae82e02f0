"""The allocation-free sort entry point (static device scratch) against the
workspace entry point, through the C-ABI: bit-identical cell_start, perm and
sorted velocities on two calls in a row, the second smaller (the scratch
keeps the first call's contents), and the size limits rejected on the
host."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_21244_amd import _lib
    _lib.load()
    return torch.device("cuda:0")


def _case(api, dev, pop, dtype):
    cell_of = torch.as_tensor(pop.cell_of, device=dev)
    v_in = torch.as_tensor(pop.v, dtype=dtype, device=dev).contiguous()
    cs_ref, perm_ref, v_ref = api.sort_cells(cell_of, pop.n_cells, v_in)
    n = pop.n
    cs = torch.full((pop.n_cells + 1,), -7, dtype=torch.int32, device=dev)
    perm = torch.full((max(n, 1),), -7, dtype=torch.int32, device=dev)
    v_out = torch.full_like(v_in, float("nan"))
    st = api.new_status(dev)
    api.sort_cells_noalloc(cell_of, pop.n_cells, v_in, cs, perm, v_out, st=st)
    torch.cuda.synchronize()
    assert torch.equal(cs, cs_ref)
    assert torch.equal(perm[:n], perm_ref)
    assert torch.equal(v_out, v_ref)
    ref = np.argsort(pop.cell_of, kind="stable")
    assert np.array_equal(perm[:n].cpu().numpy(), ref)
    return api.read_status(st)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_sort_matches_workspace_sort(dev, dtype):
    from paper_2602_21244_amd import api
    print("noalloc sort", dtype, flush=True)
    # the largest case the static scratch allows, then a smaller ragged one
    big = W.cavity_grid(seed=3, nx=200, ny=200)
    assert big.n <= 1 << 20
    _case(api, dev, big, dtype)
    small = W.ragged_population(5, 300, 90)
    _case(api, dev, small, dtype)


def test_noalloc_sort_rejects_beyond_limits(dev):
    from paper_2602_21244_amd import api
    L = api.L
    print("noalloc sort limits", flush=True)
    lib = api.lib()
    vz = L.Vec3()
    rc = lib.dsmc_sort_cells_noalloc((1 << 20) + 1, 10, None, L.F32, vz, vz, None, None, None,
                                     None)
    assert rc == L.DSMC_E_ARG and b"static scratch" in lib.dsmc_last_error()
    rc = lib.dsmc_sort_cells_noalloc(10, (1 << 20) + 1, None, L.F32, vz, vz, None, None, None,
                                     None)
    assert rc == L.DSMC_E_ARG
