"""The C-ABI library loads and exports every entry point include/rkmi.h declares
(no GPU needed: nothing is computed)."""
import ctypes
import os
import re

from .conftest import ROOT


def _declared():
    with open(os.path.join(ROOT, "include", "rkmi.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rk_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for want in ("rk_integrate_rkck", "rk_integrate_rkc", "rk_adjoint_rkc", "rk_problem_create_vdp",
                 "rk_problem_create_mass_action", "rk_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_1611_02274_amd import _lib
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_calls():
    """Calls that touch no device: version, problem handles, dims, errors."""
    import paper_1611_02274_amd as rk
    assert rk.version() >= 100
    p = rk.Problem.vdp()
    assert (p.n_eq, p.n_param, p.n_theta) == (2, 1, 1)
    q = rk.Problem.network(rk.inputs.standard_network(13))
    assert (q.n_eq, q.n_param, q.n_theta) == (13, 2, 27)
    L = rk._lib.lib()
    assert L.rk_problem_create_vdp(None) == rk._lib.RK_EINVAL
    assert b"NULL" in L.rk_last_error()


def test_batch_create_host_only():
    """A batch handle is found for the compiled set of networks in any order and
    refused for a set without a compiled batch kernel (no device touched)."""
    import ctypes as C

    import paper_1611_02274_amd as rk
    nets = [rk.inputs.standard_network(k) for k in (53, 9, 32, 13)]
    b = rk.Batch([rk.Problem.network(n) for n in nets])
    assert b._h
    L = rk._lib.lib()
    two = [rk.Problem.network(n) for n in nets[:2]]
    arr = (C.c_void_p * 2)(*[p.handle.value for p in two])
    h = C.c_void_p()
    assert L.rk_batch_create(arr, 2, C.byref(h)) == rk._lib.RK_EUNSUPPORTED
    vdp = rk.Problem.vdp()
    arr1 = (C.c_void_p * 1)(vdp.handle.value)
    assert L.rk_batch_create(arr1, 1, C.byref(h)) == rk._lib.RK_EINVAL


def test_cost_order_workspace_host_only():
    """The cost order's workspace follows the integration's own (plain schedule
    of a register-held network: none) at 256-byte alignment: pilot statistics
    (6 int32 rows), the order map, a 4096-bucket histogram and its offsets."""
    import ctypes as C

    import paper_1611_02274_amd as rk
    from paper_1611_02274_amd import _lib
    L = _lib.lib()
    p = rk.Problem.network(rk.inputs.standard_network(13))
    a256 = lambda x: (x + 255) // 256 * 256  # noqa: E731
    for n in (1, 65, 1000, 262144):
        o = rk._options(schedule=1)
        assert L.rk_workspace_bytes(p.handle, _lib.RK_METHOD_RKC, n, C.byref(o)) == 0
        o = rk._options(schedule=1, cost_order=1)
        want = a256(6 * 4 * n) + a256(4 * n) + 2 * a256(4096 * 4)
        assert L.rk_workspace_bytes(p.handle, _lib.RK_METHOD_RKC, n, C.byref(o)) == want
    # max_steps, four int32 fields, cost_order, sr_method, group_align, reserved[3]: the
    # struct keeps its size
    assert C.sizeof(_lib.Options) == 8 + 4 * 4 + 4 + 4 * 5 == 48
