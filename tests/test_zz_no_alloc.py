"""The allocation-free solve (lse_solve_static), through the C ABI, against
the workspace entry points (lse_init + lse_run + lse_mask / lse_lsf on a
caller-owned workspace): two calls in a row on one GPU, the second on a
smaller image, each equal bit for bit to its own workspace run.  Both paths
run the same kernels in the same workspace layout, so the binary results and
the LSF must be identical, not merely close."""
import numpy as np
import pytest

from paper_1409_7474_amd import lse, synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _workspace_run(p, img, mask, iters, stop, dev, stream):
    nbytes = lse.lse_workspace_bytes(p)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
    ctx = lse.lse_init(p, img.data_ptr(), mask.data_ptr(), ptr, nbytes, stream)
    lse.lse_run(ctx, iters, stop, stream)
    m = torch.empty(tuple(mask.shape), dtype=torch.uint8, device=dev)
    f = torch.empty(tuple(mask.shape), dtype=torch.float32, device=dev)
    lse.lse_mask(ctx, m.data_ptr(), stream)
    lse.lse_lsf(ctx, f.data_ptr(), stream)
    torch.cuda.synchronize(dev)
    lse.lse_destroy(ctx)
    return m.cpu().numpy(), f.cpu().numpy()


def _static_run(p, img, mask, iters, stop, dev, stream):
    m = torch.empty(tuple(mask.shape), dtype=torch.uint8, device=dev)
    f = torch.empty(tuple(mask.shape), dtype=torch.float32, device=dev)
    lse.lse_solve_static(p, img.data_ptr(), mask.data_ptr(), iters, stop, m.data_ptr(), f.data_ptr(), stream)
    return m, f


def _inputs(dev, h, w, bands, seed):
    sc = synth.scene_multiband(seed, size=max(h, w), bands=bands, n_roofs=8, n_roads=2, height=h, width=w)
    return (torch.tensor(np.asarray(sc.image, np.float32), device=dev),
            {"region": torch.tensor(sc.init_region, dtype=torch.uint8, device=dev),
             "edge": torch.tensor(sc.init_edge, dtype=torch.uint8, device=dev)})


CASES = [
    # term, bands, storage, order, reinit_every, TS, (big shape), (small shape), iterations
    ("region", 4, "f32", "table1", 1, 7, (600, 700), (230, 301), 40),
    ("edge", 4, "f32", "table1", 1, 11, (512, 640), (200, 261), 30),
    ("region", 1, "f16", "listing", 2, 9, (300, 400), (128, 150), 20),
    ("region_intensity", 3, "bf16", "table1", 3, 7, (320, 256), (97, 130), 20),
]


@pytest.mark.parametrize("term,bands,storage,order,every,ts,big,small,iters", CASES)
def test_static_solve_equals_workspace_solve_twice(dev, term, bands, storage, order, every, ts, big, small, iters):
    stream = torch.cuda.Stream(dev)
    sid = int(stream.cuda_stream)
    runs = []
    for seed, (h, w) in ((1, big), (2, small)):
        img, masks = _inputs(dev, h, w, bands, seed)
        p = lse.make_params(h, w, bands, term=term, order=order, sigma=1.0 + 0.25 * (ts // 2 - 3), ksize=ts,
                            storage=storage, reinit_every=every)
        assert lse.lse_workspace_bytes(p) <= lse.STATIC_WORKSPACE_BYTES
        mask = masks["edge" if term == "edge" else "region"]
        runs.append((p, img, mask))
    # inputs were written on the current stream: the solve stream waits for them
    stream.wait_stream(torch.cuda.current_stream(dev))
    print(f"static solve: {term} B={bands} {storage} {order} every {every} TS {ts}: {big} then {small}",
          flush=True)
    refs = [_workspace_run(p, img, mask, iters, False, dev, sid) for p, img, mask in runs]
    # Two calls in a row in the library's one array: the second, smaller
    # image finds the first call's contents there.
    outs = [_static_run(p, img, mask, iters, False, dev, sid) for p, img, mask in runs]
    torch.cuda.synchronize(dev)
    for (m_ref, f_ref), (m, f) in zip(refs, outs):
        np.testing.assert_array_equal(m.cpu().numpy(), m_ref)
        np.testing.assert_array_equal(f.cpu().numpy().view(np.uint32), f_ref.view(np.uint32))
        assert 0 < m_ref.sum() < m_ref.size


def test_static_solve_stops_when_unchanged_like_run(dev):
    """Step 5: with stop_when_unchanged the static solve ends at the same
    fixed point as lse_run, after a larger call left its state behind."""
    stream = torch.cuda.Stream(dev)
    sid = int(stream.cuda_stream)
    big_img, big_masks = _inputs(dev, 700, 500, 4, 3)
    stream.wait_stream(torch.cuda.current_stream(dev))
    pb = lse.make_params(700, 500, 4, sigma=1.0, ksize=7)
    # its outputs stay referenced until the stream has written them (a freed
    # tensor's memory could otherwise be handed to the next inputs meanwhile)
    big_out = _static_run(pb, big_img, big_masks["region"], 25, False, dev, sid)
    torch.cuda.synchronize(dev)
    del big_out
    img = torch.full((200, 240, 1), 0.3, dtype=torch.float32, device=dev)
    img[60:130, 80:150] = 0.7
    mask = torch.zeros((200, 240), dtype=torch.uint8, device=dev)
    mask[50:150, 60:180] = 1
    p = lse.make_params(200, 240, 1, sigma=1.0, ksize=7)
    stream.wait_stream(torch.cuda.current_stream(dev))  # inputs written on the current stream
    m_ref, f_ref = _workspace_run(p, img, mask, 200, True, dev, sid)
    m, f = _static_run(p, img, mask, 200, True, dev, sid)
    torch.cuda.synchronize(dev)
    np.testing.assert_array_equal(m.cpu().numpy(), m_ref)
    np.testing.assert_array_equal(f.cpu().numpy().view(np.uint32), f_ref.view(np.uint32))
    exact = np.zeros((200, 240), np.uint8)
    exact[60:130, 80:150] = 1
    np.testing.assert_array_equal(m_ref, exact)


def test_static_solve_rejects_oversized_images(dev):
    p = lse.make_params(2100, 2100, 4)  # 16.25 B/px: about 72 MB of workspace
    assert lse.lse_workspace_bytes(p) > lse.STATIC_WORKSPACE_BYTES
    x = torch.zeros(1, device=dev)
    with pytest.raises(lse.LSEError) as e:
        lse.lse_solve_static(p, x.data_ptr(), x.data_ptr(), 1, False, x.data_ptr())
    assert e.value.status == lse.LSE_ERR_WORKSPACE
