"""The C-ABI library loads, exports every symbol declared in include/pfl.h,
and its host-side validation returns the documented error codes.  Nothing
here launches GPU work (pfl_query_sizes is host-only)."""
import ctypes as C
import math
import os
import re

import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(pfl_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    import paper_2407_01651_amd as pfl
    lib = C.CDLL(pfl.LIB_PATH)
    decl = _declared()
    assert len(decl) >= 12
    for n in decl:
        assert hasattr(lib, n), n


def test_binding_covers_declared_symbols():
    import paper_2407_01651_amd as pfl
    assert set(_declared()) <= set(pfl.EXPORTED)


def _code(w, store=None):
    import paper_2407_01651_amd as pfl
    p = pfl.make_params(w, store)
    s = pfl.Sizes()
    return pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)), s


def test_sizes_of_the_coupled_workload():
    import paper_2407_01651_amd as pfl
    w = workloads.get("coupled2d_128")
    rc, s = _code(w)
    assert rc == 0
    N = 128 * 128
    assert s.pops_bytes == (9 + 5 + 5 + 5 + 5) * N * 8
    assert s.hist_bytes == (2 + 2 + 2 + 2) * N * 8
    assert s.macros_bytes == 9 * N * 8
    assert s.state_bytes == (29 + 8) * N * 8
    rc, s16 = _code(w, "f16")
    assert rc == 0 and s16.pops_bytes == 29 * N * 2 and s16.hist_bytes == 8 * N * 4


@pytest.mark.parametrize("change,code", [
    (dict(nu_l=-0.1), -1),                       # viscosity < 0: rate outside (0, 2)
    (dict(M_phi=0.0), -1),
    (dict(PeD=-1.0), -1),
    (dict(k=1.5), -1),
    (dict(nx=2), -1),
    (dict(fields=("ns", "phi", "psi", "c")), -2),   # isothermal + bubbles + solute
    (dict(dim=3, nz=8, phi_q=9), -2),             # phi on 9 velocities in 3D
    (dict(phi_q=7), -1),
    (dict(delta_n2=0.0), -1),
    (dict(th_cp_g=0.0), -1),                     # heat property ratios must be positive
    (dict(th_k_g=-1.0), -1),
])
def test_invalid_parameters_are_rejected(change, code):
    w = workloads.get("coupled2d_128")
    w.update(change)
    rc, _ = _code(w)
    assert rc == code


def test_error_message_is_thread_local_text():
    import paper_2407_01651_amd as pfl
    w = workloads.get("coupled2d_128")
    w["nu_g"] = -1.0
    rc, _ = _code(w)
    assert rc == -1
    assert "viscosit" in pfl._lib.pfl_last_error().decode()


def test_bad_rounding_mode_is_rejected():
    import paper_2407_01651_amd as pfl
    w = workloads.get("coupled2d_128")
    p = pfl.make_params(w, "f16", "nearest")
    assert p.rounding == 1
    p.rounding = 7
    s = pfl.Sizes()
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == -1
    assert "rounding" in pfl._lib.pfl_last_error().decode()



def test_write_policy_values():
    import paper_2407_01651_amd as pfl
    w = workloads.get("coupled2d_128")
    s = pfl.Sizes()
    for name, code in (("auto", 0), ("cached", 1), ("stream", 2)):
        p = pfl.make_params(dict(w, write_policy=name))
        assert p.write_policy == code
        assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == 0
    p.write_policy = 3
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == -1
    assert "write policy" in pfl._lib.pfl_last_error().decode()


def test_boundary_flags():
    """wall[a]: 0 periodic, 1 walls, 2 symmetry planes, 3 / 4 a symmetry plane
    on the low / high side only, 5 / 6 a far-field high side with a wall /
    symmetry plane low, 7 velocity sides on both ends, 8 / 9 a velocity side
    on the high / low side with a wall on the other, 10 / 11 a velocity side
    on the low / high side with a pressure side on the other (2D flow without
    the gas phase); anything else is rejected."""
    import paper_2407_01651_amd as pfl
    w = workloads.get("coupled2d_128")
    w["symmetric"] = (True, True, False)
    w["periodic"] = (False, False, True)
    p = pfl.make_params(w, "f64", "nearest")
    assert list(p.wall) == [2, 2, 0]
    s = pfl.Sizes()
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == 0
    w["symmetric"] = ("lo", "hi", False)
    p = pfl.make_params(w, "f64", "nearest")
    assert list(p.wall) == [3, 4, 0]
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == 0
    w["symmetric"] = ("lo", False, False)
    w["farfield"] = ("hi", "hi", False)
    p = pfl.make_params(w, "f64", "nearest")
    assert list(p.wall) == [6, 5, 0]
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == 0
    p.wall[0] = 12
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == -1
    assert "boundary" in pfl._lib.pfl_last_error().decode()
    p.wall[0] = 7                    # velocity sides with the gas phase active
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == pfl.E_UNSUPPORTED
    assert "gas phase" in pfl._lib.pfl_last_error().decode()
    wv = workloads.small(nx=20, ny=30, fields=("ns", "psi", "theta"), periodic=(False, False, True))
    wv.update(symmetric=(True, False, False), velocity=(False, True, False), v_in=(0.0, 0.01, 0.0))
    p = pfl.make_params(wv, "f64", "nearest")
    assert list(p.wall) == [2, 7, 0] and list(p.v_in) == [0.0, 0.01, 0.0]
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == 0
    wv.update(symmetric=(False, False, False), velocity=(False, "hi", False))
    assert list(pfl.make_params(wv).wall) == [1, 8, 0]
    wv["velocity"] = (False, "lo", False)
    assert list(pfl.make_params(wv).wall) == [1, 9, 0]
    wv["outflow"] = (False, "hi", False)
    assert list(pfl.make_params(wv).wall) == [1, 10, 0]
    wv.update(velocity=(False, "hi", False), outflow=(False, "lo", False))
    p11 = pfl.make_params(wv)
    assert list(p11.wall) == [1, 11, 0]
    assert pfl._lib.pfl_query_sizes(C.byref(p11), C.byref(s)) == 0
    wv["outflow"] = (False, "hi", False)
    with pytest.raises(ValueError):
        pfl.make_params(wv)
    wv["outflow"] = (False, False, False)
    p.v_in[1] = float("nan")
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == -1
    wv["symmetric"] = (False, True, False)
    with pytest.raises(ValueError):
        pfl.make_params(wv)
    w["farfield"] = ("lo", False, False)
    with pytest.raises(ValueError):
        pfl.make_params(w, "f64", "nearest")
    w3 = workloads.get("coupled3d_256")
    w3["periodic"] = (True, False, True)
    w3["symmetric"] = (False, "lo", False)
    w3["farfield"] = (False, "hi", False)
    p = pfl.make_params(w3, "f16", "stochastic")
    assert list(p.wall) == [0, 6, 0]
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == 0


def _declarations_with_comments():
    """(name, comment text before the declaration) for every function
    declared in include/*.h."""
    out = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        last = 0
        for m in re.finditer(r"^\s*(?:int|int64_t|const char\*)\s+(pfl_\w+)\s*\(", txt, re.M):
            out.append((m.group(1), txt[last:m.start()]))
            last = txt.index(";", m.end()) + 1
    return out


def test_every_declared_function_cites_its_passage():
    """Each entry point's comment names the passage of the paper that defines
    the operation, or says that the operation is not in the paper; the
    allocation-free variant names the callers it is for instead."""
    cite = re.compile(r"Sec\. \d|Appendix [AB]|not in the paper|no paper passage|does not treat|"
                      r"callers that cannot allocate")
    decl = _declarations_with_comments()
    assert len(decl) >= 20
    missing = [n for n, c in decl if not cite.search(c)]
    assert not missing, missing


def test_abi_version_and_parameter_struct():
    import paper_2407_01651_amd as pfl
    h = open(os.path.join(ROOT, "include", "pfl.h")).read()
    assert f"#define PFL_ABI_VERSION {pfl.ABI_VERSION}" in h
    w = workloads.get("coupled2d_128")
    p = pfl.make_params(dict(w, reduce_every=50))
    assert p.reduce_every == 50
    s = pfl.Sizes()
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == 0
    p.reduce_every = -1
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == -1
    assert "reduce_every" in pfl._lib.pfl_last_error().decode()


def test_host_argument_checks_of_new_entry_points():
    """Null contexts and bad masks are rejected on the host, before any GPU
    work (no context is created here)."""
    import paper_2407_01651_amd as pfl
    lib = pfl._lib
    assert lib.pfl_get_macros(None, 0, None, 0) == -1
    assert lib.pfl_adjoint_seed(None, None, 1, None) == -1
    assert lib.pfl_last_check(None, None) == -1
    assert lib.pfl_init_from_macros(None, None, 0, None, 0) == -1


def test_aac_form_parameter():
    import paper_2407_01651_amd as pfl
    w = workloads.get("coupled2d_128")
    s = pfl.Sizes()
    assert pfl.make_params(w).aac_form == 0
    p = pfl.make_params(dict(w, aac_form="le1"))
    assert p.aac_form == 1
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == 0
    p.aac_form = 2
    assert pfl._lib.pfl_query_sizes(C.byref(p), C.byref(s)) == -1
    assert "AAC form" in pfl._lib.pfl_last_error().decode()
