"""Host-side checks of the C ABI: the library loads, exports every function
include/gv.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2607_02749_amd import gv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gv_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gv_query_sizes", "gv_state_create", "gv_state_destroy", "gv_apply_ansatz",
                     "gv_energy", "gv_energy_grad", "gv_pauli_sum_create",
                     "gv_pauli_sum_prepare", "gv_pauli_sum_destroy", "gv_batch_energy_grad",
                     "gv_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = gv.lib()
    missing = [name for name in declared_functions() if not hasattr(L, name)]
    assert not missing, missing


def test_version_and_num_params():
    L = gv.lib()
    assert b"gv" in L.gv_version()
    a = gv.Ansatz(28, 6).c()
    assert L.gv_num_params(ctypes.byref(a)) == 336
    a = gv.Ansatz(8, 4, gv.ENT_CNOT_CIRCULAR, 1).c()
    assert L.gv_num_params(ctypes.byref(a)) == 2 * 8 * 5   # Eq. 8
    bad = gv.Ansatz(0, 1).c()
    assert L.gv_num_params(ctypes.byref(bad)) == -1


def test_query_sizes():
    sb, wb = gv.query_sizes(gv.Ansatz(28, 6), "c64", "fused", "uncompute")
    assert sb == 8 << 28
    assert wb >= 8 << 28                       # holds the adjoint vector
    _, wck = gv.query_sizes(gv.Ansatz(28, 6), "c64", "fused", "checkpoint")
    assert wck >= wb + 4 * (8 << 28)           # states after layers 1..4 (layer 0 is regenerated)
    # store: one buffer per tile pass but the last; at n = 28 the snake order
    # runs 3 passes for layer 1 and 2 for each of layers 2..5 (two-layer
    # passes at every boundary), so 11 passes -> 10 buffers
    _, wst = gv.query_sizes(gv.Ansatz(28, 6), "c64", "fused", "store")
    assert wst - wb == 10 * (8 << 28)
    # CNOT ladders keep the layer boundaries only
    _, wcn = gv.query_sizes(gv.Ansatz(20, 5, ent=3), "c64", "fused", "store")
    _, wcn_ck = gv.query_sizes(gv.Ansatz(20, 5, ent=3), "c64", "fused", "checkpoint")
    assert wcn == wcn_ck
    sb128, _ = gv.query_sizes(gv.Ansatz(10, 2), "c128", "plain")
    assert sb128 == 16 << 10
    _, _, db = gv.query_sizes(gv.Ansatz(28, 6), "c64", "fused", "store", with_diag=True)
    assert db == 8 << 28                       # FP64 diagonal
    with pytest.raises(gv.GVError):
        gv.query_sizes(gv.Ansatz(35, 1))
    with pytest.raises(gv.GVError):
        gv.query_sizes(gv.Ansatz(10, 1, ent=9))


def test_state_create_validation():
    L = gv.lib()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: creation only records it
    assert L.gv_state_create(10, 0, 0, None, 1 << 20, None, 0, None, ctypes.byref(h)) == 1
    assert L.gv_state_create(10, 0, 0, fake, 100, None, 0, None, ctypes.byref(h)) == 2
    assert L.gv_state_create(0, 0, 0, fake, 1 << 20, None, 0, None, ctypes.byref(h)) == 1
    assert L.gv_state_create(10, 7, 0, fake, 1 << 20, None, 0, None, ctypes.byref(h)) == 1
    misaligned = ctypes.c_void_p((1 << 20) + 8)
    assert L.gv_state_create(10, 0, 0, misaligned, 1 << 20, None, 0, None, ctypes.byref(h)) == 1
    assert b"aligned" in L.gv_last_error()
    assert L.gv_state_create(10, 0, 0, fake, 1 << 20, None, 0, None, ctypes.byref(h)) == 0
    # calls that validate before enqueueing anything
    a = gv.Ansatz(11, 1).c()
    assert L.gv_apply_ansatz(h, fake, ctypes.byref(a)) == 4       # n mismatch
    a = gv.Ansatz(10, 1).c()
    assert L.gv_apply_ansatz(h, None, ctypes.byref(a)) == 1       # NULL params
    e = ctypes.c_void_p(2 << 20)
    assert L.gv_energy(h, None, e) == 1
    assert L.gv_state_destroy(h) == 0


def test_pauli_sum_merge_and_groups():
    n = 4
    x = [0, 0, 0b0011, 0b0011, 0b0100, 0b1000, 0]
    z = [0b0001, 0b0001, 0, 0b0011, 0b0100, 0, 0]
    c = [0.5, 0.25, 1.0, 2.0, 3.0, 0.0, 1.5]
    h = gv.PauliSum(n, x, z, c)
    nd, no, ng = h.info()
    assert nd == 2          # Z0 merged (0.75) and the identity
    assert no == 3          # XX on (0,1), YY on (0,1), Y on 2 (X on 3 has c = 0)
    assert ng == 2          # {XX, Y2} commute qubit-wise, YY needs its own group
    with pytest.raises(gv.GVError):
        gv.PauliSum(n, [0], [1 << 4], [1.0])          # mask bit >= n
    with pytest.raises(gv.GVError):
        gv.PauliSum(n, [0], [1], [float("nan")])


def test_pauli_sum_groups_of_generated_workload():
    from paper_2607_02749_amd import synth
    w = synth.make_instance(32, 1, 10, 2, 32, seed=0, m_off=2000,
                            off_types=("XX", "YY", "XZ", "ZY"), off_groups=64)
    h = gv.PauliSum(32, w.x, w.z, w.c)
    nd, no, ng = h.info()
    assert no == 2000 and ng <= 64


def test_batch_call_validates_before_any_gpu_work():
    L = gv.lib()
    fake = ctypes.c_void_p(1 << 20)    # never dereferenced: validation fails first
    arr = (gv._Instance * 1)()
    cl = (gv._Cluster * 1)()
    arr[0].ansatz = gv.Ansatz(12, 2).c()
    arr[0].params_dev = None
    arr[0].h = None
    assert L.gv_batch_energy_grad(1, arr, cl, 0, fake, 1 << 20, None, fake, fake) == 1
    h = gv.PauliSum(12, [0], [1], [1.0])
    arr[0].params_dev = 1 << 20
    arr[0].h = h.handle
    # Hamiltonian not prepared
    assert L.gv_batch_energy_grad(1, arr, cl, 0, fake, 1 << 20, None, fake, fake) == 4
    arr[0].ansatz = gv.Ansatz(8, 2).c()
    assert L.gv_batch_energy_grad(1, arr, cl, 0, fake, 1 << 20, None, fake, fake) == 3
    assert L.gv_batch_energy_grad(-1, arr, cl, 0, fake, 1 << 20, None, fake, fake) == 1


def test_cover_plan_of_n32_workload():
    # 2,000 two-qubit XX/YY/XZ/ZY terms on 32 qubits: tiles of 12 index bits
    # keep the 4 low bits, so each pass holds 8 more; the planner must cover
    # every term, stage at most 512 per pass, and use far fewer passes than
    # one per pair of qubits
    from paper_2607_02749_amd import synth
    w = synth.workload_n32()
    h = gv.PauliSum(32, w.x, w.z, w.c)
    passes, most, loose = h.plan("c64")
    print("n=32 cover passes", passes, "most terms in a pass", most, "loose", loose)
    assert loose == 0
    assert most <= 512
    assert passes <= 24
    # tiny registers run on the plain engine: every term one by one
    h2 = gv.PauliSum(6, [3, 5], [0, 1], [1.0, 0.5])
    assert h2.plan("c128") == (0, 0, 2)
