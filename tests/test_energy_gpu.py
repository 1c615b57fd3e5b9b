"""GPU parity of the energy diagnostics (1/2 sum |u|^2, 1/2 sum |curl A|^2 over
the interior, FP64, deterministic) against the CPU oracle, through the C ABI."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2406_08923_amd import inputs

torch = pytest.importorskip("torch")
import paper_2406_08923_amd as S  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def load(plan, bufs, vals, dtype):
    """Put the interior values (rounded to the storage type) with periodic
    halos into the plan's buffers; return the rounded padded FP64 arrays."""
    out = []
    for k, v in enumerate(vals):
        t = torch.from_numpy(O.pad_periodic(v, 3)).cuda().to(bufs[k].dtype)
        plan.padded(bufs[k]).copy_(t)
        out.append(plan.padded(bufs[k]).to(torch.float64).cpu().numpy())
    return out


@pytest.mark.parametrize("prec", [S.PREC_F64, S.PREC_F32_MASTER64, S.PREC_BF16_MASTER64])
@pytest.mark.parametrize("n", [(37, 29, 23), (64, 8, 5), (3, 3, 3)])
def test_energy_matches_oracle(prec, n):
    f, _ = inputs.fourier_fields(n, 5, nf=8, modes=4, kmax=3, amp=0.3)
    plan = S.RkPlan(S.MODEL_MHD8, n, prec)
    bufs = plan.alloc()["f_a"]
    rounded = load(plan, bufs, f, prec)
    ds = [2 * math.pi / v for v in n]
    want = O.energy(rounded, ds)
    got = plan.energy(bufs)
    assert np.allclose(got, want, rtol=1e-12, atol=0), (got, want)
    again = plan.energy(bufs)
    assert np.array_equal(got, again)  # fixed partition and tree: bitwise repeatable


def test_energy_pitched_layout_and_after_a_step():
    n = (33, 26, 21)
    f, _ = inputs.fourier_fields(n, 6, nf=8, modes=4, kmax=3, amp=0.3)
    plan = S.RkPlan(S.MODEL_MHD_FULL, n, S.PREC_F64, row_pitch=64, x_offset=16)
    b = plan.alloc()
    for k in range(8):
        b["f_a"][k].fill_(float("nan"))  # columns outside the padded field are never read
    load(plan, b["f_a"], f, S.PREC_F64)
    ds = [2 * math.pi / v for v in n]
    dt = 0.05 * min(ds)
    res = plan.run(b["f_a"], b["f_b"], b["w"], 1, dt)  # f_out with valid halos
    pads = [plan.padded(t).cpu().numpy() for t in res]
    want = O.energy(pads, ds)
    assert np.allclose(plan.energy(res), want, rtol=1e-12, atol=0)


def test_energy_of_a_single_potential_mode():
    # A_z = a cos(k x): 1/2 sum |B|^2 = a^2 keff^2 N / 4 (sixth-order symbol)
    n = (32, 8, 6)
    x = 2 * math.pi * np.arange(n[0]) / n[0]
    a, k = 0.5, 3
    vals = [np.zeros(n[::-1]) for _ in range(8)]
    vals[7] = np.broadcast_to(a * np.cos(k * x), n[::-1]).copy()
    plan = S.RkPlan(S.MODEL_MHD8, n, S.PREC_F64)
    bufs = plan.alloc()["f_a"]
    load(plan, bufs, vals, S.PREC_F64)
    h = 2 * math.pi / n[0]
    keff = 2 / h * (0.75 * math.sin(k * h) - 0.15 * math.sin(2 * k * h) + math.sin(3 * k * h) / 60)
    N = n[0] * n[1] * n[2]
    ek, em = plan.energy(bufs)
    assert ek == 0.0
    assert math.isclose(em, a * a * keff * keff * N / 4, rel_tol=1e-12)


def test_energy_rejects_non_mhd_plans():
    plan = S.RkPlan(S.MODEL_ADVDIFF, (16, 16, 16), S.PREC_F64)
    bufs = plan.alloc()["f_a"] * 8
    with pytest.raises(S.StencilError):
        plan.energy(bufs)
