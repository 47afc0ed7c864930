"""Full-size checks in the launch configuration the benchmark times.

n = 28 (complex64, L = 6, 20,000 Z-strings): the energy and the whole
gradient against the oracle's values stored in tests/golden/oracle_n28.json
(written by tests/golden/make_golden.py from the oracle alone), for the
uncompute and store gradient modes.

n = 32 (complex64, 32 GiB per state): the oracle cannot run here, so the
checks are properties that hold at any size: with no entangler the state is
a product state and E and its gradient have a closed form (Bloch vectors,
product rule) for the n = 32 Hamiltonian, including its off-diagonal
groups; with the CZ ladder the three memory modes must agree."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import closed_forms as cf  # noqa: E402
from paper_2607_02749_amd import gv, synth  # noqa: E402

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-30))


def evaluate(inst, precision, mode):
    an = gv.Ansatz(inst.n, inst.layers, inst.ent, inst.final_rotation)
    st = gv.State(inst.n, precision, "fused", an, mode)
    h = gv.PauliSum(inst.n, inst.x, inst.z, inst.c).prepare(st)
    th = torch.tensor(inst.theta, dtype=torch.float64, device=st.device)
    e, g = gv.energy_grad(st, h, th, an, None, mode)
    torch.cuda.synchronize()
    out = e.cpu().numpy(), g.cpu().numpy()
    del st, h, th, e, g
    torch.cuda.empty_cache()
    return out


def test_n28_diagonal_entries_against_stored_oracle():
    # 16 seeded entries of the FP64 diagonal, each a direct sum over the
    # 20,000 Z-strings in the oracle (tests/golden/make_golden.py)
    gold = json.load(open(os.path.join(HERE, "golden", "oracle_n28.json")))
    inst = synth.workload_n28()
    h = gv.PauliSum(inst.n, inst.x, inst.z, inst.c).prepare_for("c64", "fused")
    d = h.diagonal()
    idx = torch.tensor(gold["diag_index"], dtype=torch.int64, device=d.device)
    got = d[idx].cpu().numpy()
    want = np.array(gold["diag_value"])
    scale = np.abs(inst.c).sum()
    print("n=28 diagonal entries: max abs err / sum|c|", np.abs(got - want).max() / scale,
          flush=True)
    assert np.abs(got - want).max() <= 1e-12 * scale
    del h, d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", ["uncompute", "store"])
def test_n28_against_stored_oracle(mode):
    gold = json.load(open(os.path.join(HERE, "golden", "oracle_n28.json")))
    inst = synth.workload_n28()
    e, g = evaluate(inst, "c64", mode)
    e_ref, g_ref = gold["energy"][0], np.array(gold["grad"])
    print(mode, "E rel", abs(e[0] - e_ref) / abs(e_ref), "grad rel L2", rel(g, g_ref), flush=True)
    assert abs(e[0] - e_ref) <= 1e-5 * abs(e_ref)
    assert rel(g, g_ref) <= 1e-4


def test_n32_product_state_closed_form():
    base = synth.workload_n32()
    inst = synth.Instance(n=32, layers=base.layers, ent=synth.ENT_NONE, final_rotation=0,
                          x=base.x, z=base.z, c=base.c, theta=base.theta)
    e_cf, g_cf = cf.product_energy_grad(inst.n, inst.layers, inst.theta, inst.x, inst.z, inst.c)
    e, g = evaluate(inst, "c64", "uncompute")
    print("n=32 product state: E", e[0], "closed form", e_cf, "grad rel L2", rel(g, g_cf),
          flush=True)
    assert abs(e[0] - e_cf) <= 1e-5 * max(abs(e_cf), 1e-3 * np.abs(inst.c).sum())
    assert rel(g, g_cf) <= 1e-4


def test_n32_memory_modes_agree():
    inst = synth.workload_n32()
    e_u, g_u = evaluate(inst, "c64", "uncompute")
    for mode in ("checkpoint", "recompute"):
        e, g = evaluate(inst, "c64", mode)
        print("n=32", mode, "E", e[0], "vs uncompute", e_u[0], "grad rel L2", rel(g, g_u),
              flush=True)
        assert abs(e[0] - e_u[0]) <= 1e-5 * abs(e_u[0])
        assert rel(g, g_u) <= 1e-4
