"""The access-pattern probe (fargo_hbm_streams, a measurement aid beside the
step): every written field equals in[q] + in[-1] element by element, in both
walking orders, on a mesh whose columns do not fill the last workgroup; the
fields past nout are left alone; overlapping outputs are refused."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


@pytest.mark.parametrize("march", [0, 1])
@pytest.mark.parametrize("nin,nout", [(1, 1), (8, 7), (9, 8), (9, 9), (3, 1)])
def test_streams_probe_writes_the_sum(march, nin, nout):
    import torch
    from paper_1602_02359_amd import fargo as F
    nx, ny, nz = 100, 7, 5  # 700 columns: the last of three workgroups is ragged
    print("probe march=%d nin=%d nout=%d" % (march, nin, nout), flush=True)
    g = torch.Generator(device="cpu").manual_seed(10 * nin + nout)
    ins = [torch.randn(nx * ny * nz, generator=g, dtype=torch.float64).cuda() for _ in range(nin)]
    outs = [torch.full((nx * ny * nz,), -7.0, dtype=torch.float64, device="cuda") for _ in range(nin)]
    F.fargo_hbm_streams(ins, outs[:nout], nx, ny, nz, march)
    torch.cuda.synchronize()
    for q in range(nin):
        if q < nout:
            assert torch.equal(outs[q], ins[q] + ins[-1]), q
        else:
            assert bool((outs[q] == -7.0).all()), q


def test_streams_probe_refuses_overlap():
    import torch
    from paper_1602_02359_amd import fargo as F
    a = torch.zeros(64, dtype=torch.float64, device="cuda")
    b = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FargoError) as e:
        F.fargo_hbm_streams([a, b], [a], 8, 8, 1, 0)
    assert e.value.code == -1
    c = torch.zeros(64, dtype=torch.float64, device="cuda")
    for outs, march in (([b], 1), ([c, c], 0)):  # an output on an input, two outputs on one buffer
        with pytest.raises(F.FargoError) as e:
            F.fargo_hbm_streams([a, b], outs, 8, 8, 1, march)
        assert e.value.code == -1
