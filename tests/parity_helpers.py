"""Shared helpers of the GPU parity tests (comparison with the FP64 oracle)."""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle

torch = pytest.importorskip("torch")

LSF_TOL = 1e-5
MASK_TOL = 1e-4


def _as_gpu(img, dev, dtype=torch.float32):
    t = torch.tensor(img, dtype=dtype, device=dev)
    return t, t.float().cpu().double().numpy()


def _make(dev, img, mask, **kw):
    from paper_1409_7474_amd import lse
    return lse.LSE(img, torch.tensor(mask, dtype=torch.uint8, device=dev), **kw)


def one_step(job, img64, *, term="region", dt=15.0, sigma=1.0, ts=7, g=None, tau=None):
    """Advance the GPU one iteration and compare with the oracle from the
    GPU's own LSF.  The binary result must match the oracle's everywhere
    except where the oracle's |u| is below tau (default 1e-5 max(1, dt), a
    sign FP32 cannot decide like FP64); at most max(4, 1e-4 N) such decisions
    may differ, and the LSF must match within 1e-5 outside their Gaussian
    footprint.  Returns (max LSF error, differing decisions, oracle result)."""
    phi = job.lsf().cpu().double().numpy()
    ref = oracle.step(phi, img64 if term == "region" else None, term=term, dt=dt, sigma=sigma, ts=ts, g=g)
    job.step()
    got = job.lsf().cpu().double().numpy()
    band = np.abs(ref.u) < (1e-5 * max(1.0, dt) if tau is None else tau)
    bits = job.mask().cpu().numpy().astype(bool)
    differ = bits != (ref.b > 0)
    wrong = differ & ~band
    assert not wrong.any(), f"{int(wrong.sum())} binary decisions differ outside the ambiguity band"
    amb = differ & band
    assert amb.sum() <= max(4, 1e-4 * amb.size), int(amb.sum())
    excl = ndi.binary_dilation(amb, structure=np.ones((ts, ts), bool)) if amb.any() else amb
    err = float(np.abs(got - ref.phi)[~excl].max()) if (~excl).any() else 0.0
    return err, int(amb.sum()), ref


def check_normaliser(st, img64, ref_M):
    """The normaliser of eq. (17) must be the maximum of |D| over every pixel.
    Recompute that maximum in FP64 from the GPU's own FP32 means; the GPU's
    value (a pruned block scan for B > 1) may differ only by the FP32
    rounding of D, bounded by 12 u * sum_b |a_b| (2 max|I_b| + |m_b|).  The
    oracle's M (FP64 means) must agree within the effect of rounding the means
    themselves to FP32 on that same scale."""
    nb = img64.shape[2]
    cp = np.array(st["c_plus"][:nb], np.float32)
    cm = np.array(st["c_minus"][:nb], np.float32)
    a32 = (cp - cm).astype(np.float64)
    m32 = (cp + cm).astype(np.float64)
    D = np.zeros(img64.shape[:2])
    for b in range(nb):
        D += a32[b] * (2.0 * img64[:, :, b] - m32[b])
    M64 = float(np.abs(D).max())
    amax = np.abs(img64).reshape(-1, nb).max(0)
    scale = float(np.sum(np.abs(a32) * (2.0 * amax + np.abs(m32))))
    assert abs(st["M"] - M64) <= 12 * 2.0 ** -24 * scale + 1e-30, (st["M"], M64, scale)
    cscale = float(np.sum((np.abs(cp) + np.abs(cm)) * (2.0 * amax + np.abs(m32))))
    assert abs(st["M"] - ref_M) <= 12 * 2.0 ** -24 * (scale + cscale), (st["M"], ref_M)


def mask_disagreement(a, b):
    return float(np.mean(a.astype(bool) != b.astype(bool)))




def round_storage(a, storage):
    """Values as the library stores them: float32, then rounded to nearest
    (ties to even) in the storage type ("f32", "f16" or "bf16"); float64 out."""
    f = np.asarray(a, dtype=np.float32)
    if storage == "f16":
        f = f.astype(np.float16).astype(np.float32)
    elif storage == "bf16":
        u = f.view(np.uint32).astype(np.uint64)
        f = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32).view(np.float32)
    return f.astype(np.float64)


def iou(a, b):
    a, b = np.asarray(a, bool), np.asarray(b, bool)
    u = np.logical_or(a, b).sum()
    return 1.0 if u == 0 else float(np.logical_and(a, b).sum() / u)
