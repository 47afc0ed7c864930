"""GPU parity for rotation angles outside [-pi, pi] (Sec. IV-B, Eq. 7-8).

The tile passes rotate a pair by RY's half angle phi = theta / 2 as three
shears, which needs cos phi >= 0: a gate with cos phi < 0 is rotated by
phi - pi instead (the same gate times -1), and the product of those signs is
carried by the generated first layer.  The other parity tests draw theta in
[-pi, pi], where no gate flips; these draw it from [-4 pi, 4 pi], add the
boundary angles +-pi, 2 pi, 3 pi, and make the number of flipped gates odd,
so that a wrong sign of the whole state would show in the amplitudes and a
sign mismatch between the forward state and lam in the gradients.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2607_02749_amd import gv, synth  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {"c128": (1e-10, 1e-10), "c64": (1e-5, 1e-4)}


def n_flipped(inst) -> int:
    """RY gates of the rotated layers (1 .. R-1) whose half angle has a
    negative cosine."""
    n, rot = inst.n, inst.layers + inst.final_rotation
    th = np.asarray(inst.theta).reshape(rot, 2, n)
    return int(np.sum(np.cos(0.5 * th[1:, 0, :]) < 0.0))


def wide(inst, seed):
    """inst with theta ~ U(-4 pi, 4 pi), a few boundary angles, and an odd
    number of flipped gates."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(-4 * np.pi, 4 * np.pi, size=inst.num_params)
    n = inst.n
    th[0] = np.pi                      # layer 0 (generated, never rotated)
    th[2 * n + 0] = np.pi              # half angle pi/2: cos > 0 in FP64, kept
    th[2 * n + 1] = -np.pi
    th[2 * n + 2] = 2 * np.pi          # half angle pi: flipped
    th[2 * n + 3] = 3 * np.pi          # half angle 3 pi / 2: cos < 0, flipped
    out = dataclasses.replace(inst, theta=th)
    if n_flipped(out) % 2 == 0:        # toggle one gate between flipped and kept
        th[2 * n + 4] = 0.5 * np.pi if np.cos(0.5 * th[2 * n + 4]) < 0.0 else 2.5 * np.pi
        out = dataclasses.replace(inst, theta=th)
    assert n_flipped(out) % 2 == 1
    return out


@pytest.mark.parametrize("precision", ["c128", "c64"])
@pytest.mark.parametrize("ent,final", [(synth.ENT_CZ_LINEAR, 0), (synth.ENT_CZ_LINEAR, 1),
                                       (synth.ENT_CNOT_LINEAR, 0)])
def test_wide_angle_amplitudes(precision, ent, final):
    inst = wide(synth.make_instance(14, 4, 10, 2, 2, seed=5, ent=ent, final_rotation=final), 1)
    an = gv.Ansatz(inst.n, inst.layers, inst.ent, inst.final_rotation)
    st = gv.State(inst.n, precision, "fused", an)
    th = torch.tensor(inst.theta, dtype=torch.float64, device="cuda")
    st.apply_ansatz(th, an)
    psi = st.amplitudes().cpu().numpy().astype(np.complex128)
    ref = oracle.prepare(inst.n, inst.layers, inst.ent, inst.theta, inst.final_rotation)
    err = np.abs(psi - ref).max()
    print(precision, ent, final, "flipped", n_flipped(inst), "max amplitude error", err,
          flush=True)
    assert err < (1e-12 if precision == "c128" else 2e-6)


@pytest.mark.parametrize("precision,mode", [("c128", "uncompute"), ("c64", "uncompute"),
                                            ("c64", "checkpoint"), ("c64", "recompute"),
                                            ("c64", "store")])
def test_wide_angle_energy_grad(precision, mode):
    inst = wide(synth.make_instance(14, 5, 150, 4, 3, seed=8, m_off=12), 2)
    an = gv.Ansatz(inst.n, inst.layers, inst.ent, inst.final_rotation)
    st = gv.State(inst.n, precision, "fused", an, mode)
    h = gv.PauliSum(inst.n, inst.x, inst.z, inst.c).prepare(st)
    th = torch.tensor(inst.theta, dtype=torch.float64, device="cuda")
    e, g = gv.energy_grad(st, h, th, an, None, mode)
    torch.cuda.synchronize()
    e, g = e.cpu().numpy(), g.cpu().numpy()
    e_ref, g_ref = oracle.energy_grad(inst.n, inst.layers, inst.ent, inst.theta, inst.x,
                                      inst.z, inst.c, final_rotation=inst.final_rotation)
    te, tg = TOL[precision]
    rel_e = abs(e[0] - e_ref.real) / abs(e_ref.real)
    rel_g = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    max_g = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print(precision, mode, "flipped", n_flipped(inst), "E rel", rel_e, "grad rel L2", rel_g,
          "max entry", max_g, flush=True)
    assert rel_e <= te and rel_g <= tg and max_g <= tg


@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_wide_angle_batch(precision):
    insts = [wide(inst, 10 + i) for i, inst in
             enumerate(synth.workload_batch(count=6, seed=4, n_lo=12, n_hi=14))]
    items = []
    for inst in insts:
        an = gv.Ansatz(inst.n, inst.layers, inst.ent, inst.final_rotation)
        th = torch.tensor(inst.theta, dtype=torch.float64, device="cuda")
        items.append((an, th, gv.PauliSum(inst.n, inst.x, inst.z, inst.c), inst.cluster_mask))
    # n = 14 instances as whole-GPU tile passes, the others in the persistent kernel
    b = gv.Batch(items, precision, graph=False, split_n=14)
    b.run()
    torch.cuda.synchronize()
    te, tg = TOL[precision]
    for i, inst in enumerate(insts):
        mask = oracle.param_mask(inst.n, inst.layers, inst.cluster_mask)
        e_ref, g_ref = oracle.energy_grad(inst.n, inst.layers, inst.ent, inst.theta, inst.x,
                                          inst.z, inst.c, mask=mask)
        e = b.energies[i].cpu().numpy()
        g = b.grads[i].cpu().numpy()
        rel_g = np.linalg.norm(g - g_ref) / max(np.linalg.norm(g_ref), 1e-30)
        print(i, inst.n, "flipped", n_flipped(inst), "E rel",
              abs(e[0] - e_ref.real) / abs(e_ref.real), "grad rel", rel_g, flush=True)
        assert abs(e[0] - e_ref.real) <= te * abs(e_ref.real)
        assert rel_g <= tg
