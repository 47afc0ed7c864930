"""GPU parity of the measurement calls (Sec. IV-F, Sec. V-A) against the
oracle's plain versions on the same amplitudes (the oracle's state, copied
to the device) and the same uniform draws: Born-rule samples (exact where
the draw is not within rounding of a cumulative-sum boundary, otherwise a
valid index), the most probable bitstring, and the finite-shot energy
estimate with its groups."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import measure as M  # noqa: E402
from paper_2607_02749_amd import gv, synth  # noqa: E402

pytestmark = pytest.mark.gpu


def device_state(psi, precision):
    dt = torch.complex64 if precision == "c64" else torch.complex128
    return torch.tensor(psi, dtype=dt, device="cuda").contiguous()


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 11, 14, 17])
def test_samples_match_inverse_cdf(n, precision):
    inst = synth.make_instance(n, 2, n, 3, 2, seed=900 + n, ent=synth.ENT_CZ_LINEAR)
    psi = oracle.prepare(n, 2, inst.ent, inst.theta)
    amps = device_state(psi, precision)
    ref_psi = amps.cpu().numpy().astype(np.complex128)     # the same numbers the GPU reads
    u = np.random.default_rng(n).random(5000)
    b = gv.sample(amps, torch.tensor(u, device="cuda")).cpu().numpy().astype(np.uint64)
    want = M.born_sample(ref_psi, u)
    p = np.abs(ref_psi) ** 2
    cdf = np.cumsum(p)
    target = u * cdf[-1]
    lo = np.concatenate([[0.0], cdf[:-1]])[b.astype(np.int64)]
    hi = cdf[b.astype(np.int64)]
    tol = 1e-12 * cdf[-1]
    # every draw is a valid inverse-CDF index ...
    assert np.all((lo - tol <= target) & (target <= hi + tol))
    assert np.all(p[b.astype(np.int64)] > 0)
    # ... and equals the oracle's wherever the target is clear of a boundary
    near = (np.abs(target - lo) < tol) | (np.abs(target - hi) < tol)
    assert np.array_equal(b[~near], want[~near])
    assert near.sum() <= 2


@pytest.mark.parametrize("precision", ["c128", "c64"])
def test_argmax_decoding(precision):
    # a peaked state: the basis state b slightly rotated
    n = 15
    from oracle import closed_forms as cf
    th = cf.basis_theta(n, 2, 0b101100111000101) + 0.05
    psi = oracle.prepare(n, 2, synth.ENT_CZ_LINEAR, th)
    amps = device_state(psi, precision)
    idx, prob = gv.argmax(amps)
    ref = amps.cpu().numpy().astype(np.complex128)
    assert int(idx.item()) == M.argmax(ref)
    assert prob.item() == pytest.approx(np.abs(ref[M.argmax(ref)]) ** 2, rel=1e-15)
    # ties: two equal largest entries -> the smaller index
    t = np.zeros(1 << 12, dtype=np.complex128)
    t[[7, 3001, 40]] = [0.6, 0.6j, 0.52]
    i2, _ = gv.argmax(device_state(t, precision))
    assert int(i2.item()) == 7


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("n", [10, 13])
def test_energy_shots_matches_oracle(n, precision):
    inst = synth.make_instance(n, 2, 10 * n, 4, 3, seed=950 + n, m_off=3 * n,
                               off_types=("XX", "YY", "XZ", "ZY"))
    psi = oracle.prepare(n, 2, inst.ent, inst.theta)
    amps = device_state(psi, precision)
    ref_psi = amps.cpu().numpy().astype(np.complex128)
    h = gv.PauliSum(n, inst.x, inst.z, inst.c).prepare_for(precision, "fused")
    groups = gv.pauli_groups(h)
    ref_groups = M.qwc_groups(inst.x, inst.z, inst.c)
    assert [(g[0], g[1], g[2], g[3]) for g in groups] == \
        [(g[0], g[1], g[2], len(g[3])) for g in ref_groups]
    shots = 8192
    u = np.random.default_rng(n).random((1 + len(groups)) * shots)
    e = gv.energy_shots(h, amps, torch.tensor(u, device="cuda"), shots).cpu().numpy()
    want = M.energy_shots(n, ref_psi, inst.x, inst.z, inst.c, u, shots,
                          single=precision == "c64")
    print(precision, "n", n, "shots estimate", e[0], "oracle", want, flush=True)
    # the same draws on the same amplitudes (rotated in the state's precision)
    # give the same samples; the sums differ only in rounding order
    assert abs(e[0] - want) <= 1e-10 * np.abs(inst.c).sum()
    # and the estimate is near the exact energy (8192 shots per group)
    exact = oracle.energy(n, 2, inst.ent, inst.theta, inst.x, inst.z, inst.c).real
    assert abs(e[0] - exact) <= 8 * np.abs(inst.c).sum() / np.sqrt(shots)
