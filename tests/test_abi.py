"""The C ABI library loads and exports every entry point the header declares;
argument validation needs no GPU."""

import os
import re

import numpy as np
import pytest

from conftest import ROOT


def _declared():
    txt = open(os.path.join(ROOT, "include", "rt_tddft.h")).read()
    return sorted(set(re.findall(r"^(?:rt_status|void|const char\*)\s+(rt_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_boundary_calls():
    names = _declared()
    for n in ("rt_init", "rt_apply_h", "rt_step", "rt_dipole", "rt_workspace_size", "rt_free", "rt_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2410_09189_amd import rt

    for n in _declared():
        assert hasattr(rt.lib, n), n


def _args(**over):
    import synth
    from rt_helpers import run_args, system_args

    s = synth.make_system(16, 0.4, 2, 2, 2, seed=1, nl_rank=4, region=(0.3, 0.7))
    psi = synth.lowpass_orbitals(16, 0.4, 4, 1)
    rp = synth.RunParams(dt=0.05, n_steps=10)
    sa = system_args(s, psi)
    ra = run_args(rp)
    for k, v in over.items():
        if hasattr(sa.struct, k):
            setattr(sa.struct, k, v)
        else:
            setattr(ra.struct, k, v)
    return sa, ra


def test_workspace_size_is_positive_and_grows_with_history():
    from paper_2410_09189_amd import rt

    sa, ra = _args()
    a = rt.rt_workspace_size([sa], ra)
    sa, ra = _args(n_steps_max=1000)
    b = rt.rt_workspace_size([sa], ra)
    assert a > 4 * 16 ** 3 * 8 and b > a


@pytest.mark.parametrize("field,value", [("h", -1.0), ("nl_rank", 3), ("max_scf", 0), ("dt", 0.0),
                                          ("n_images", 9), ("precision", 7), ("hupdate", 5)])
def test_invalid_arguments_are_rejected(field, value):
    from paper_2410_09189_amd import rt

    sa, ra = _args(**{field: value})
    with pytest.raises(rt.RTError) as e:
        rt.rt_workspace_size([sa], ra)
    assert e.value.status == rt.RT_EINVAL
    assert rt.rt_last_error()


def test_projector_wider_than_cell_rejected():
    from paper_2410_09189_amd import rt

    sa, ra = _args(nl_rcut=4.0)
    with pytest.raises(rt.RTError):
        rt.rt_workspace_size([sa], ra)


def test_mixed_precision_grid_limit_rejected():
    """BF16x3 kernels address a 128-row tile with 32-bit byte offsets: 2^23 points and
    above are refused before any allocation."""
    from paper_2410_09189_amd import rt

    sa, ra = _args(precision=rt.RT_MIXED)
    sa.struct.n[0], sa.struct.n[1], sa.struct.n[2] = 256, 256, 128
    with pytest.raises(rt.RTError) as e:
        rt.rt_workspace_size([sa], ra)
    assert e.value.status == rt.RT_EINVAL
    assert "2^23" in rt.rt_last_error()


@pytest.mark.parametrize("over", [dict(nonorthogonal=1, orthonormalize=1), dict(nonorthogonal=1, magnus_order=4)])
def test_nonorthogonal_basis_exclusions_rejected(over):
    """A non-orthogonal basis is exclusive with orthonormalisation and is not
    combined with the second Magnus term."""
    from paper_2410_09189_amd import rt

    sa, ra = _args(**over)
    with pytest.raises(rt.RTError) as e:
        rt.rt_workspace_size([sa], ra)
    assert e.value.status == rt.RT_EINVAL
    assert "nonorthogonal" in rt.rt_last_error() or "orthonormal basis" in rt.rt_last_error()


@pytest.mark.parametrize("jump,mask", [((16, 0, 0), 0), ((0, -1, 0), 1), ((0, 0, 0), 8), ((0, 0, 0), -1)])
def test_sawtooth_jump_and_dipole_mask_checked(jump, mask):
    """The jump plane must lie on the grid and the correction mask select axes only."""
    from paper_2410_09189_amd import rt

    sa, ra = _args(dipole_correction=mask)
    sa.struct.saw_jump[:] = list(jump)
    with pytest.raises(rt.RTError) as e:
        rt.rt_workspace_size([sa], ra)
    assert e.value.status == rt.RT_EINVAL
    assert "saw_jump" in rt.rt_last_error() or "dipole_correction" in rt.rt_last_error()


def test_dipole_correction_adds_its_partial_sums():
    from paper_2410_09189_amd import rt

    sa, ra = _args()
    a = rt.rt_workspace_size([sa], ra)
    sa, ra = _args(dipole_correction=5)
    sa.struct.saw_jump[:] = [3, 15, 0]
    b = rt.rt_workspace_size([sa], ra)
    assert b > a


@pytest.mark.parametrize("over", [dict(h_block=4, hupdate=0), dict(h_block=4, hupdate=1, orthonormalize=1),
                                  dict(h_block=-1, hupdate=1)])
def test_h_block_needs_the_local_update_and_given_orthonormal_orbitals(over):
    """Blocked initialisation never holds H applied to every orbital, which the full
    update and the library's orthonormalisation need."""
    from paper_2410_09189_amd import rt

    sa, ra = _args(**over)
    with pytest.raises(rt.RTError) as e:
        rt.rt_workspace_size([sa], ra)
    assert e.value.status == rt.RT_EINVAL and ("h_block" in rt.rt_last_error())


def test_h_block_shrinks_the_workspace():
    from paper_2410_09189_amd import rt

    sa, ra = _args(hupdate=1)
    a = rt.rt_workspace_size([sa], ra)
    sa, ra = _args(hupdate=1, h_block=1)
    b = rt.rt_workspace_size([sa], ra)
    assert a - b == 3 * 16 ** 3 * 8  # N = 4: the H Psi buffer holds 1 orbital instead of 4


def test_fp64_full_updates_hold_one_h_psi_buffer_per_trajectory():
    """FP64 full updates of several trajectories keep every trajectory's H Psi, so
    that one projection launch covers them: the workspace grows by T N ng doubles
    over the local update's, and not at all for a single trajectory."""
    import synth
    from rt_helpers import run_args

    from paper_2410_09189_amd import rt

    sa, _ = _args()
    rp = synth.RunParams(dt=0.05, n_steps=10)
    w = {(len(ax), h): rt.rt_workspace_size([sa], run_args(rp, n_traj_axes=ax, hupdate=h))
         for ax in ((0,), (0, 1, 2)) for h in (0, 1)}
    assert w[(1, 0)] == w[(1, 1)]
    assert w[(3, 0)] - w[(3, 1)] == 3 * 4 * 16 ** 3 * 8  # T = 3, N = 4, 16^3 points


def test_fp64_full_update_h_psi_buffers_stop_at_16_gib():
    """Past 16 GiB the trajectories' H Psi share one buffer (64 orbitals on 128^3:
    16 trajectories take exactly 16 GiB, 17 would take more)."""
    import synth
    from rt_helpers import run_args

    from paper_2410_09189_amd import rt

    rp = synth.RunParams(dt=0.05, n_steps=10)
    w = {}
    for t in (16, 17):
        for h in (0, 1):
            sa, _ = _args(n_virt=62)
            sa.struct.n[0] = sa.struct.n[1] = sa.struct.n[2] = 128
            assert sa.struct.n_occ + sa.struct.n_virt == 64
            w[(t, h)] = rt.rt_workspace_size([sa], run_args(rp, n_traj_axes=[q % 3 for q in range(t)], hupdate=h))
    assert w[(16, 0)] - w[(16, 1)] == 16 << 30
    assert w[(17, 0)] == w[(17, 1)]


def test_nonorthogonal_basis_takes_overlap_buffers():
    from paper_2410_09189_amd import rt

    sa, ra = _args()
    a = rt.rt_workspace_size([sa], ra)
    sa, ra = _args(nonorthogonal=1)
    b = rt.rt_workspace_size([sa], ra)
    assert b >= a + 3 * 4 * 4 * 8  # overlap, its inverse and S^-1 Hbar per trajectory (N = 4)


def test_ground_state_and_eigh_reject_bad_arguments_without_a_gpu():
    import synth
    from paper_2410_09189_amd import rt
    from rt_helpers import system_args

    s = synth.make_system(16, 0.4, 2, 2, 2, seed=1, nl_rank=4, region=(0.3, 0.7))
    sa = system_args(s, synth.lowpass_orbitals(16, 0.4, 4 + 6, 1))
    size = rt.rt_ground_state_workspace_size(sa, rt.gs_params(n_guard=6))
    assert size > 3 * 10 * 16 ** 3 * 8
    bad = [dict(n_guard=1), dict(n_guard=1100), dict(degree=0), dict(degree=65), dict(max_scf=0),
           dict(max_passes=0), dict(tol_rho=0.0), dict(tol_res=-1.0), dict(mix=0.0), dict(mix=1.5),
           dict(pulay_depth=0), dict(pulay_depth=9)]
    for kw in bad:
        p = rt.gs_params(**{"n_guard": 6, **kw})
        with pytest.raises(rt.RTError) as e:
            rt.rt_ground_state_workspace_size(sa, p)
        assert e.value.status == rt.RT_EINVAL, kw
        with pytest.raises(rt.RTError) as e:  # rejected before any device work
            rt.rt_ground_state(sa, p, 0, 0, 0, 0)
        assert e.value.status == rt.RT_EINVAL, kw
    sa.struct.orthonormalize = 1
    with pytest.raises(rt.RTError):
        rt.rt_ground_state_workspace_size(sa, rt.gs_params(n_guard=6))
    sa.struct.orthonormalize = 0
    with pytest.raises(rt.RTError) as e:
        rt.rt_ground_state(sa, rt.gs_params(n_guard=6), 0, size, 0, 0)
    assert e.value.status == rt.RT_EINVAL and "NULL" in rt.rt_last_error(None)
    assert rt.rt_eigh_workspace_size(255) >= 3 * 256 * 256 * 8
    for n in (0, 4097):
        with pytest.raises(rt.RTError):
            rt.rt_eigh_workspace_size(n)
    with pytest.raises(rt.RTError) as e:
        rt.rt_eigh(0, 8, 0, 0, 0, 0, 1 << 20)
    assert e.value.status == rt.RT_EINVAL


def test_binding_refuses_orbital_arrays_of_the_wrong_size():
    """The library reads N (rt_init) or N + n_guard (rt_ground_state) orbitals from
    psi0; the binding refuses shorter or wrongly typed arrays before any device work."""
    import synth
    from paper_2410_09189_amd import rt
    from rt_helpers import run_args, system_args

    s = synth.make_system(16, 0.4, 2, 2, 2, seed=1, nl_rank=4, region=(0.3, 0.7))
    short = synth.lowpass_orbitals(16, 0.4, 3, 1)  # N = 4 needed
    with pytest.raises(ValueError):
        rt.rt_init([system_args(s, short)], run_args(synth.RunParams(dt=0.05, n_steps=2)), 0, 0, 0)
    exact = synth.lowpass_orbitals(16, 0.4, 4, 1)  # N rows, but the ground state needs N + n_guard
    with pytest.raises(ValueError):
        rt.ground_state(system_args(s, exact), rt.gs_params(n_guard=6))
    sa = system_args(s, exact)
    sa.psi0 = exact.astype(np.float32)
    with pytest.raises(ValueError):
        rt.rt_init([sa], run_args(synth.RunParams(dt=0.05, n_steps=2)), 0, 0, 0)


def test_eigh_noalloc_rejects_sizes_beyond_its_static_array_without_a_gpu():
    """The allocation-free eigensolver refuses n outside [1, RT_EIGH_NOALLOC_MAX_N]
    and NULL pointers before touching a device."""
    from paper_2410_09189_amd import rt

    txt = open(os.path.join(ROOT, "include", "rt_tddft.h")).read()
    assert int(re.search(r"#define RT_EIGH_NOALLOC_MAX_N (\d+)", txt).group(1)) == rt.RT_EIGH_NOALLOC_MAX_N
    for n in (0, -3, rt.RT_EIGH_NOALLOC_MAX_N + 1, 4096):
        with pytest.raises(rt.RTError) as e:
            rt.rt_eigh_noalloc(0, n, 8, 8, 8)
        assert e.value.status == rt.RT_EINVAL
        assert "outside" in rt.rt_last_error(None)
    with pytest.raises(rt.RTError) as e:
        rt.rt_eigh_noalloc(0, 8, 0, 8, 8)
    assert e.value.status == rt.RT_EINVAL and "NULL" in rt.rt_last_error(None)


def test_checkpoint_calls_refuse_null_contexts_without_a_gpu():
    import ctypes

    from paper_2410_09189_amd import rt

    n = ctypes.c_size_t(0)
    assert rt.lib.rt_checkpoint_size(None, ctypes.byref(n)) == rt.RT_EINVAL
    buf = (ctypes.c_char * 16)()
    assert rt.lib.rt_checkpoint_save(None, buf, 16) == rt.RT_EINVAL
    assert rt.lib.rt_checkpoint_load(None, buf, 16) == rt.RT_EINVAL
