"""The binding refuses outputs and workspaces that are not in the input's GPU
memory.  The library takes bare pointers: a host tensor's address handed to
a kernel would be a memory fault rather than an error, so every such buffer
is checked on the host before the call (nothing here reaches a kernel)."""
import numpy as np
import pytest

from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return torch_cuda()


@pytest.fixture(scope="module")
def cw():
    from paper_2408_14302_amd import cwth
    return cwth


def test_host_and_mistyped_buffers_are_refused(torch, cw):
    n = 5000
    x = torch.randn(n, device="cuda")
    p = cw.Plan(16000.0, [1.0, 8.0], 4, "bf16")
    K = p.num_frames(n)
    bad_outs = [torch.empty(2, K), torch.empty(2, K, dtype=torch.float64, device="cuda"),
                torch.empty(2, K + 1, device="cuda"), torch.empty(K, 2, device="cuda").t()]
    for o in bad_outs:
        with pytest.raises(ValueError):
            p.execute(x, o)
        with pytest.raises(ValueError):
            cw.execute_batch([p], [x], [o])
        with pytest.raises(ValueError):
            cw.Batch(4)([p], [x], [o])
    assert p.output(n).is_cuda
    with pytest.raises(ValueError):
        cw.decimate(x, 2, out=torch.empty(cw.decimated_length(n, 2)))
    with pytest.raises(TypeError):
        cw.decimate(x, 2, h=torch.ones(1))
    w = p(x)
    ws = int(cw.raw().cwt_image_workspace_bytes())
    with pytest.raises(ValueError):
        cw.scalogram_image(w, 8, 8, out=torch.empty(8, 8))
    with pytest.raises(ValueError):
        cw.scalogram_image(w, 8, 8, workspace=torch.empty(ws, dtype=torch.uint8))
    with pytest.raises(ValueError):
        cw.scalogram_image(w, 8, 8, workspace=torch.empty(ws // 2, dtype=torch.uint8, device="cuda"))
    h = cw.daubechies(2)
    with pytest.raises(ValueError):
        cw.dwt_scalogram(x, h, 3, pyramid=torch.empty(cw.dwt_pyramid_length(n, 3)))
    with pytest.raises(ValueError):
        cw.dwt_scalogram(x, h, 3, out=torch.empty(3, n))
    # the same calls with device buffers run
    out = p.output(n)
    p.execute(x, out)
    img = cw.scalogram_image(w, 8, 8, out=torch.empty(8, 8, device="cuda"),
                             workspace=torch.empty(ws, dtype=torch.uint8, device="cuda"))
    S, pyr = cw.dwt_scalogram(x, h, 3, out=torch.empty(3, n, device="cuda"),
                              pyramid=torch.empty(cw.dwt_pyramid_length(n, 3), device="cuda"))
    torch.cuda.synchronize()
    assert torch.equal(out, w)
    assert float(img.min()) >= 0.0 and float(img.max()) <= 1.0
    assert tuple(S.shape) == (3, n)
