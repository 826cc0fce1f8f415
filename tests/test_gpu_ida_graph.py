"""The IDA loop replayed as a HIP graph (ida_graph_create / ida_graph_launch)
gives, on every replay, exactly what the eager ida_refine gives with the same
arguments.  Replays are interleaved with eager library work and host
synchronisation, and every replay is checked, because a graph that is right
on its first replay only is the failure mode to rule out."""
import numpy as np
import pytest

import synth

from gpu_util import Run, pack_images, device

pytestmark = pytest.mark.gpu


def _setup():
    imgs = [synth.synth_image(31, 64, 64), synth.synth_image(32, 48, 80)]
    px, d = pack_images(imgs)
    entries = [dict(d[0], block=16, subrate=0.25, method="dd"), dict(d[1], block=16, subrate=0.2, method="bbv")]
    return Run(px, entries).budget().sense()


@pytest.mark.parametrize("denoiser,iters", [("identity", 4), ("bm3d", 3), ("cnn", 3)])
def test_graph_replays_match_eager(denoiser, iters):
    import torch
    import paper_2001_09632_amd as g
    from oracle import cnn as ocnn
    dev = device()
    run = _setup()
    plan = run.plan
    params = None
    if denoiser == "cnn":
        # a narrow accepted range, so that the BM3D fallback runs inside the
        # graph for the images whose sigma leaves it
        params = torch.from_numpy(g.denoiser_params(ocnn.init_params(5), (1.0, 150.0))).to(dev)
    nbytes = g.ida_workspace_bytes(plan, denoiser)

    def bufs():
        return (torch.full((plan.pixels,), float("nan"), dtype=torch.float32, device=dev),
                torch.full((iters * plan.n,), float("nan"), dtype=torch.float32, device=dev),
                torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev))

    x_e, tr_e, ws_e = bufs()
    g.ida_refine(plan, run.y, run.k, run.off, x_e, iters, 2.0, denoiser, params=params, sigma_trace=tr_e,
                 workspace=ws_e)
    torch.cuda.synchronize()
    ref_x, ref_tr = x_e.cpu().numpy().copy(), tr_e.cpu().numpy().copy()
    assert np.all(np.isfinite(ref_x)) and np.all(np.isfinite(ref_tr))

    x_g, tr_g, ws_g = bufs()
    graph = g.IdaGraph(plan, run.y, run.k, run.off, x_g, iters, 2.0, denoiser, params=params,
                       sigma_trace=tr_g, workspace=ws_g)
    try:
        for rep in range(3):
            x_g.fill_(float("nan"))
            tr_g.fill_(float("nan"))
            graph.launch()
            # eager work of the same kind between replays
            x2, tr2, ws2 = bufs()
            g.ida_refine(plan, run.y, run.k, run.off, x2, iters, 2.0, denoiser, params=params,
                         sigma_trace=tr2, workspace=ws2)
            torch.cuda.synchronize()
            assert np.array_equal(x_g.cpu().numpy(), ref_x), f"replay {rep}: x differs"
            assert np.array_equal(tr_g.cpu().numpy(), ref_tr), f"replay {rep}: sigma trace differs"
            assert np.array_equal(x2.cpu().numpy(), ref_x)
    finally:
        graph.close()


def test_graph_bad_arguments():
    import torch
    import paper_2001_09632_amd as g
    dev = device()
    run = _setup()
    x = torch.empty(run.plan.pixels, dtype=torch.float32, device=dev)
    ws = torch.empty(16, dtype=torch.uint8, device=dev)
    with pytest.raises(g.AbcsError, match="ENOSPACE"):
        g.IdaGraph(run.plan, run.y, run.k, run.off, x, 2, 2.0, "bm3d", workspace=ws)
    with pytest.raises(g.AbcsError, match="EDOMAIN"):
        g.IdaGraph(run.plan, run.y, run.k, run.off, x, 2, 0.5, "identity", workspace=ws)
