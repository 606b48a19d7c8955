"""The access-pattern reference (mhs_probe_smoother_pattern) writes what its
contract says and nothing else: with u_in = 0 every interior node of u_out
equals f (the added multiple of the loaded sum is zero), every boundary
node keeps its previous value, for both tiles, several z-chunk lengths and
requests per launch, on shapes with ragged tiles in every axis."""

import ctypes as C

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1307_6720_amd import _lib  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("dims", [(33, 33, 33), (257, 17, 9), (65, 129, 35)])
@pytest.mark.parametrize("tile", [0, 1])
@pytest.mark.parametrize("kz", [1, 5, 32])
@pytest.mark.parametrize("nreq", [1, 3])
def test_probe_writes_f_on_interior_nodes_only(dims, tile, kz, nreq):
    nx, ny, nz = dims
    print(f"[probe] dims {dims} tile {tile} kz {kz} nreq {nreq}", flush=True)
    g = torch.Generator().manual_seed(nx * 131 + ny * 7 + nz + tile + 10 * kz + 100 * nreq)
    n = nx * ny * nz
    u = torch.zeros(nreq * n, dtype=torch.float32, device=DEV)
    f = torch.rand(nreq * n, generator=g, dtype=torch.float32).to(DEV)
    o = torch.full((nreq * n,), -7.0, dtype=torch.float32, device=DEV)
    s = C.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    _lib.check(_lib.lib().mhs_probe_smoother_pattern(C.c_void_p(u.data_ptr()), C.c_void_p(f.data_ptr()),
                                                     C.c_void_p(o.data_ptr()), nx, ny, nz, nreq, tile, kz, s))
    torch.cuda.synchronize()
    o = o.view(nreq, nz, ny, nx).cpu()
    f = f.view(nreq, nz, ny, nx).cpu()
    interior = torch.zeros((nz, ny, nx), dtype=torch.bool)
    interior[1:-1, 1:-1, 1:-1] = True
    assert torch.equal(o[:, interior], f[:, interior])
    assert bool((o[:, ~interior] == -7.0).all())
