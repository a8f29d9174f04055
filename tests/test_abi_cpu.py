"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and
rejects invalid arguments before touching a device."""
import ctypes as C

import numpy as np
import pytest

from oracle.fem import TaylorHood
from oracle.tableau import tableau
from paper_2202_07381_amd import irkmg
from paper_2202_07381_amd import workloads as wl


def test_exports_every_declared_symbol():
    names = irkmg.header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(irkmg.lib, n), n


@pytest.mark.parametrize("fam,r", [("radauIIA", 1), ("radauIIA", 2), ("radauIIA", 3), ("gauss", 1), ("gauss", 2),
                                   ("gauss", 3), ("lobattoIIIC", 2), ("lobattoIIIC", 3)])
def test_builtin_tableaux_match_oracle(fam, r):
    A, b, c = irkmg.irk_tableau_builtin(fam, r)
    Ao, bo, co = tableau(fam, r)
    assert np.abs(A - Ao).max() < 1e-15 and np.abs(b - bo).max() < 1e-15 and np.abs(c - co).max() < 1e-15


def test_unknown_tableau_rejected():
    with pytest.raises(irkmg.IrkError) as e:
        irkmg.irk_tableau_builtin("lobattoIIIC", 1)
    assert e.value.status == irkmg.IRK_EINVAL


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_node_numbering_matches_oracle(dim):
    xyz, cells = wl.square_mesh(5) if dim == 2 else wl.cube_mesh(2)
    got = irkmg.irk_mesh_p2_nodes(wl.MeshLevel(dim, xyz, cells, None))
    assert np.array_equal(got, TaylorHood(xyz, cells).node_xyz)


def _setup_status(levels, r=2, dt=0.1, nu=1.0, opts=None, nlev=None):
    structs = []
    keep = []
    for lv in levels:
        s, k = irkmg._mesh_struct(lv)
        structs.append(s)
        keep += k
    arr = (irkmg.irk_mesh_level * max(1, len(structs)))(*structs)
    A, b, c = np.eye(max(r, 1)) * 0.5, np.ones(max(r, 1)) / max(r, 1), np.ones(max(r, 1))
    tab = irkmg.irk_tableau(r, A.ctypes.data, b.ctypes.data, c.ctypes.data)
    h = C.c_void_p()
    st = irkmg.lib.irk_mg_setup(arr, len(structs) if nlev is None else nlev, C.byref(tab), dt, nu, None,
                                C.byref(opts) if opts else None, None, C.byref(h))
    return st, irkmg.lib.irk_last_error().decode()


def test_setup_validation_before_device_work():
    lv = wl.square_hierarchy(2, 2)
    assert _setup_status(lv, r=5)[0] == irkmg.IRK_EINVAL
    assert _setup_status(lv, r=0)[0] == irkmg.IRK_EINVAL
    assert _setup_status(lv, nlev=0)[0] == irkmg.IRK_EINVAL
    assert _setup_status(lv, dt=-1.0)[0] == irkmg.IRK_EINVAL
    assert _setup_status(lv, nu=float("nan"))[0] == irkmg.IRK_EINVAL
    bad = wl.square_hierarchy(2, 2)
    bad[1].parent = None
    assert _setup_status(bad)[0] == irkmg.IRK_EINVAL
    bad = wl.square_hierarchy(2, 2)
    bad[1].parent = bad[1].parent.copy()
    bad[1].parent[3] = 10**6
    st, msg = _setup_status(bad)
    assert st == irkmg.IRK_EINVAL and "parent" in msg
    bad = wl.square_hierarchy(2, 2)
    bad[1].cells = bad[1].cells.copy()
    bad[1].cells[0, 0] = -4
    assert _setup_status(bad)[0] == irkmg.IRK_EINVAL
    # a level that is not a uniform refinement
    skip = [wl.square_hierarchy(2, 1)[0], wl.square_hierarchy(2, 3)[2]]
    assert _setup_status(skip)[0] == irkmg.IRK_EINVAL
    opts = irkmg.irk_mg_opts(2, 2, -0.5, 1, 0)
    assert _setup_status(lv, opts=opts)[0] == irkmg.IRK_EINVAL
    opts = irkmg.irk_mg_opts(2, 2, 0.5, 3, 0)
    assert _setup_status(lv, opts=opts)[0] == irkmg.IRK_EINVAL


def test_null_handle_calls_fail_cleanly():
    assert irkmg.lib.irk_mg_vcycle(None, None, None, None) == irkmg.IRK_EINVAL
    assert irkmg.lib.irk_fgmres_solve(None, None, None, 1e-8, 10, 30, None, None) == irkmg.IRK_EINVAL
    assert irkmg.lib.irk_mg_ndofs(None, -1) == -1
    irkmg.lib.irk_mg_destroy(None)


# ------------------------------------------------------------ stage eigenbasis (host)
@pytest.mark.parametrize("family,r", [("radauIIA", 1), ("radauIIA", 2), ("radauIIA", 3), ("gauss", 2),
                                      ("gauss", 3), ("lobattoIIIC", 2), ("lobattoIIIC", 3)])
def test_stage_basis_builtin(family, r):
    """A = W T W^{-1} with T real block diagonal: real eigenvalues first, then pairs as
    [[a, b], [-b, a]], b > 0; the eigenvalues agree with LAPACK's."""
    from paper_2202_07381_amd import irkmg

    A, b, c = irkmg.irk_tableau_builtin(family, r)
    W, Wi, T = irkmg.irk_stage_basis(A)
    assert np.abs(W @ T @ Wi - A).max() < 1e-13
    assert np.abs(W @ Wi - np.eye(r)).max() < 1e-13
    ev = []
    k = 0
    while k < r:
        if k + 1 < r and T[k, k + 1] != 0.0:
            a_, b_ = T[k, k], T[k, k + 1]
            assert b_ > 0 and T[k + 1, k] == -b_ and T[k + 1, k + 1] == a_
            assert np.all(T[k:k + 2, :k] == 0) and np.all(T[k:k + 2, k + 2:] == 0)
            ev += [a_ + 1j * b_, a_ - 1j * b_]
            k += 2
        else:
            assert np.count_nonzero(T[k]) <= 1
            ev.append(T[k, k])
            k += 1
    ref = np.linalg.eigvals(A)
    assert np.abs(np.sort_complex(np.array(ev)) - np.sort_complex(ref)).max() < 1e-12


def test_stage_basis_known_spectrum():
    """4x4 matrix with prescribed eigenvalues (two real, one pair) in a random basis."""
    from paper_2202_07381_amd import irkmg

    rng = np.random.default_rng(5)
    V = rng.standard_normal((4, 4))
    T0 = np.array([[0.2, 0, 0, 0], [0, 0.7, 0, 0], [0, 0, 0.3, 0.45], [0, 0, -0.45, 0.3]])
    A = V @ T0 @ np.linalg.inv(V)
    W, Wi, T = irkmg.irk_stage_basis(A)
    assert np.abs(W @ T @ Wi - A).max() < 1e-12
    assert np.allclose(np.diag(T)[:2], [0.2, 0.7], atol=1e-12)
    assert np.allclose(T[2:, 2:], T0[2:, 2:], atol=1e-12)


@pytest.mark.parametrize("A", [np.array([[1.0, 1.0], [0.0, 1.0]]),   # defective
                               2.0 * np.eye(2),                         # repeated
                               np.zeros((5, 5))])                       # r > 4
def test_stage_basis_rejects(A):
    from paper_2202_07381_amd import irkmg

    with pytest.raises(irkmg.IrkError) as ei:
        irkmg.irk_stage_basis(A)
    assert ei.value.status == irkmg.IRK_EINVAL


def test_stage_basis_gauss4():
    """The 4-stage Gauss collocation tableau (built from Gauss--Legendre nodes) has two
    complex eigenvalue pairs; the decomposition reproduces A and LAPACK's spectrum."""
    from paper_2202_07381_amd import irkmg

    x, _ = np.polynomial.legendre.leggauss(4)
    c = 0.5 * (x + 1.0)
    V = np.vander(c, 4, increasing=True)
    m = np.arange(1, 5)
    A = (c[:, None] ** m[None, :] / m[None, :]) @ np.linalg.inv(V)
    assert np.allclose(A.sum(axis=1), c, atol=1e-14)
    W, Wi, T = irkmg.irk_stage_basis(A)
    assert np.abs(W @ T @ Wi - A).max() < 1e-13
    assert T[0, 1] > 0 and T[2, 3] > 0  # two pairs
    ev = np.concatenate([[T[0, 0] + 1j * T[0, 1], T[0, 0] - 1j * T[0, 1]],
                         [T[2, 2] + 1j * T[2, 3], T[2, 2] - 1j * T[2, 3]]])
    assert np.abs(np.sort_complex(ev) - np.sort_complex(np.linalg.eigvals(A))).max() < 1e-12


def test_hessenberg_eigenvalues_against_lapack():
    """irk_hessenberg_eigs (shifted QR in complex arithmetic) against numpy's LAPACK
    eigenvalues on random upper Hessenberg matrices (real and complex-pair spectra) and
    on a block of plane rotations with a known spectrum; error paths."""
    rng = np.random.default_rng(61)
    for m in (1, 2, 5, 12, 30, 64):
        H = np.triu(rng.standard_normal((m + 1, m)), -1)
        ev = irkmg.irk_hessenberg_eigs(H, m)
        ref = np.linalg.eigvals(H[:m, :m])
        assert np.all(np.diff(ev.real) <= 1e-12)
        for z in ref:  # every LAPACK eigenvalue has a close partner
            assert np.min(np.abs(ev - z)) <= 1e-9 * max(1.0, np.abs(ref).max()), (m, z)
    R = np.zeros((6, 6))
    for k, (a, b) in enumerate([(1.0, 2.0), (-0.5, 0.25), (3.0, 1.0)]):
        R[2 * k:2 * k + 2, 2 * k:2 * k + 2] = [[a, b], [-b, a]]
    R[0, 5] = 0.7
    ev = irkmg.irk_hessenberg_eigs(R)
    want = np.array([3 + 1j, 3 - 1j, 1 + 2j, 1 - 2j, -0.5 + 0.25j, -0.5 - 0.25j])
    assert all(np.min(np.abs(ev - z)) < 1e-12 for z in want)
    with pytest.raises(irkmg.IrkError):
        irkmg.irk_hessenberg_eigs(np.zeros((3, 3)), 0)


def test_struct_layouts_match_the_header(tmp_path):
    # every ctypes structure of the binding has the size and field offsets that a C
    # compiler gives the header's struct (a field added on one side only fails here)
    import ctypes
    import shutil
    import subprocess

    from paper_2202_07381_amd import irkmg

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [irkmg.irk_mesh_level, irkmg.irk_tableau, irkmg.irk_mg_opts, irkmg.irk_solve_info,
               irkmg.irk_batch_opts, irkmg.irk_kernel_stats, irkmg.irk_newton_opts, irkmg.irk_newton_info,
               irkmg.irk_mhd_opts]
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{irkmg.MHD_HEADER}"', "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for field, _ in st._fields_:
            lines.append(f'  printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for st in structs:
        name = st.__name__
        assert int(out[name]) == ctypes.sizeof(st), name
        for field, _ in st._fields_:
            assert int(out[f"{name}.{field}"]) == getattr(st, field).offset, (name, field)
