"""Pins of the oracle's half-spectrum layout (Supplementary S1.2: real fields
keep only the non-redundant half of the transform, columns x = 0 .. nx/2;
the omitted half follows from q(-k) = conj q(k)).

What fixes the half layout independently of the oracle's own code:
* its transforms are numpy's rfftn / irfftn (a library routine, also on
  spectra whose self-conjugate columns are not Hermitian);
* the per-mode arithmetic is that of the full layout at the same k, so with
  every block active the stored coefficients equal the full layout's;
* for an exactly Hermitian state and right-hand side the candidate at -k is
  the exact conjugate of the one at k, so G over the stored half equals G
  over the full spectrum bit for bit;
* the dense trajectory of a real field is the full layout's (same physics);
* the free energy (Parseval with the omitted partners) and the mass match;
* single modes land in the documented block (columns below nx/2 first, then
  one block per (z, y) block row for the column nx/2).
"""
import numpy as np
import pytest

from paper_2609_03922_amd import inputs

CH_P, GS_P = (1.0, 1.0), (0.16, 0.08, 0.035, 0.060)


def _inst(o, op, dims, block, tau, flags, dt=None):
    p = CH_P if op == o.OP_CH else GS_P
    dt = dt if dt is not None else (0.01 if op == o.OP_CH else 1.0)
    return o.Inst(op=op, dims=dims, block=block, tau=tau, dx=1.0, dt=dt, p=p, flags=flags)


def _hermitian_half(rng, shape):
    """A random half spectrum whose columns x = 0 and x = nx/2 are exactly
    Hermitian in (z, y), so its extension is an exactly Hermitian spectrum."""
    nz, ny, nx = shape
    xs = nx // 2 + 1
    h = rng.standard_normal((nz, ny, xs)) + 1j * rng.standard_normal((nz, ny, xs))
    for ix in (0, nx // 2):
        for iz in range(nz):
            for iy in range(ny):
                jz, jy = (-iz) % nz, (-iy) % ny
                if (jz, jy) == (iz, iy):
                    h[iz, iy, ix] = h[iz, iy, ix].real
                elif (iz, iy) < (jz, jy):
                    h[jz, jy, ix] = np.conj(h[iz, iy, ix])
    return h


def _extend(h, nx):
    """Full spectrum from a half one by q(-k) = conj q(k)."""
    nz, ny, xs = h.shape
    full = np.zeros((nz, ny, nx), np.complex128)
    full[:, :, :xs] = h
    for ix in range(xs, nx):
        for iz in range(nz):
            for iy in range(ny):
                full[iz, iy, ix] = np.conj(h[(-iz) % nz, (-iy) % ny, nx - ix])
    return full


@pytest.mark.parametrize("shape", [(16, 16, 16), (1, 32, 32), (1, 1, 64)])
def test_transforms_are_numpys_rfftn_irfftn(oracle_mod, shape):
    o = oracle_mod
    rng = inputs.rng_for(71, len(shape))
    real = rng.standard_normal(shape)
    h = o.rfft(real)
    assert np.allclose(h, np.fft.rfftn(real), rtol=0, atol=1e-12 * np.abs(h).max())
    # any half spectrum, the self-conjugate columns not Hermitian
    hs = shape[:-1] + (shape[-1] // 2 + 1,)
    z = rng.standard_normal(hs) + 1j * rng.standard_normal(hs)
    got = o.irfft(z, shape)
    ref = np.fft.irfftn(z, s=shape, axes=tuple(range(len(shape))))
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    assert np.abs(o.irfft(h, shape) - real).max() <= 1e-13


def test_single_modes_land_in_their_blocks(oracle_mod):
    o = oracle_mod
    n, B = 16, 4  # stored 16 x 16 x 9; 4 x 4 x 2 blocks below x = 8, then 4 x 4 for x = 8
    inst = _inst(o, o.OP_CH, (n, n, n), (B, B, B), 1e-3, o.FLAG_HALF | o.FLAG_STATE)
    assert inst.n_blocks == 32 + 16 and inst.n_modes == n * n * 9
    for (iz, iy, ix), want in [((5, 2, 3), ((1 * 4 + 0) * 2 + 0)),
                               ((13, 9, 7), ((3 * 4 + 2) * 2 + 1)),
                               ((6, 14, 8), 32 + 1 * 4 + 3),
                               ((0, 1, 8), 32 + 0)]:
        q = np.zeros((n, n, 9), np.complex128)
        q[iz, iy, ix] = 3.0 - 4.0j
        res = o.apply(inst, q.ravel(), np.zeros(q.size, np.complex128))
        assert np.flatnonzero(res["mask"]).tolist() == [want], (iz, iy, ix)
        assert res["a_b"][want] == 25.0 and res["G"] == 25.0


def test_nyquist_column_increment_activates_its_block(oracle_mod):
    """Increment measure: a right-hand side only on the column nx/2."""
    o = oracle_mod
    n, B = 32, 8
    inst = _inst(o, o.OP_CH, (1, n, n), (1, B, B), 0.5, o.FLAG_HALF)
    q = np.zeros((n, 17), np.complex128)
    r = np.zeros_like(q)
    r[19, 16] = 2.0 + 1.0j
    res = o.apply(inst, q.ravel(), r.ravel())
    nbm = (n // B) * (n // (2 * B))
    assert np.flatnonzero(res["mask"]).tolist() == [nbm + 19 // B]
    assert res["G"] > 0 and res["a_b"][nbm + 19 // B] == res["G"]


@pytest.mark.parametrize("op,dtype", [("ch", "f64"), ("ch", "f32"), ("gs", "f64"), ("gs", "f32")])
def test_stored_coefficients_equal_the_full_layout(oracle_mod, op, dtype):
    """Every block active: the half layout updates each stored mode exactly
    as the full layout updates the same k (also the column nx/2)."""
    o = oracle_mod
    opc = o.OP_CH if op == "ch" else o.OP_GS
    shape = (16, 16, 16)
    ns = 2 if op == "gs" else 1
    rng = inputs.rng_for(72, ns)
    qf = rng.standard_normal((ns,) + shape) + 1j * rng.standard_normal((ns,) + shape)
    rf = rng.standard_normal((ns,) + shape) + 1j * rng.standard_normal((ns,) + shape)
    qh, rh = qf[..., :9], rf[..., :9]
    full = _inst(o, opc, shape, (4, 4, 4), 0.0, o.FLAG_PIN_K0)
    half = _inst(o, opc, shape, (4, 4, 4), 0.0, o.FLAG_PIN_K0 | o.FLAG_HALF)
    kw = {}
    if dtype == "f32":
        kw = dict(dtype="f32", k0=qf[:, 0, 0, 0].real.copy(), rhs_k0=rf[:, 0, 0, 0].real.copy())
    a = o.apply(full, qf.ravel(), rf.ravel(), **kw)
    b = o.apply(half, qh.ravel(), rh.ravel(), **kw)
    assert a["mask"].all() and b["mask"].all()
    qa = a["q"].reshape((ns,) + shape)[..., :9]
    assert np.array_equal(b["q"].reshape((ns,) + qh.shape[1:]), qa)
    if dtype == "f32":
        assert np.array_equal(a["k0"], b["k0"])


@pytest.mark.parametrize("op,state", [("ch", False), ("ch", True), ("gs", False)])
def test_G_over_the_stored_half_equals_the_full_G_for_hermitian_inputs(oracle_mod, op, state):
    o = oracle_mod
    opc = o.OP_CH if op == "ch" else o.OP_GS
    shape = (8, 8, 8)
    rng = inputs.rng_for(73, 1)
    ns = 2 if op == "gs" else 1
    hq = [_hermitian_half(rng, shape) for _ in range(ns)]
    hr = [_hermitian_half(rng, shape) for _ in range(ns)]
    fq = np.concatenate([_extend(h, 8).ravel() for h in hq])
    fr = np.concatenate([_extend(h, 8).ravel() for h in hr])
    fl = o.FLAG_PIN_K0 | (o.FLAG_STATE if state else 0)
    a = o.apply(_inst(o, opc, shape, (2, 2, 2), 0.85, fl), fq, fr)
    b = o.apply(_inst(o, opc, shape, (2, 2, 2), 0.85, fl | o.FLAG_HALF),
                np.concatenate([h.ravel() for h in hq]), np.concatenate([h.ravel() for h in hr]))
    assert a["G"] == b["G"] and b["G"] > 0
    assert 0 < b["count"] < b["mask"].size


@pytest.mark.parametrize("op", ["ch", "gs"])
def test_dense_half_trajectory_is_the_full_layouts(oracle_mod, op):
    o = oracle_mod
    opc = o.OP_CH if op == "ch" else o.OP_GS
    n, steps = 32, 20
    if op == "ch":
        fields = [inputs.uniform_field(1001, 7, (n, n), 0.0, 0.05)]
    else:
        u = np.ones((n, n))
        v = np.zeros((n, n))
        u[8:16, 10:18], v[8:16, 10:18] = 0.5, 0.25
        v = v + 0.01 * inputs.uniform_field(1004, 7, (n, n), 0.0, 1.0)
        fields = [u, v]
    full0 = np.concatenate([np.fft.fft2(f).ravel() for f in fields])
    half0 = np.concatenate([o.rfft(f).ravel() for f in fields])
    blk = (1, 8, 8)
    F = o.step(_inst(o, opc, (1, n, n), blk, 0.0, o.FLAG_DENSE), full0, steps)["state"]
    H = o.step(_inst(o, opc, (1, n, n), blk, 0.0, o.FLAG_DENSE | o.FLAG_HALF), half0, steps)["state"]
    ns = len(fields)
    for s in range(ns):
        rf = np.real(np.fft.ifft2(F.reshape(ns, n, n)[s]))
        rh = o.irfft(H.reshape(ns, n, n // 2 + 1)[s], (n, n))
        assert np.linalg.norm(rh - rf) <= 1e-12 * np.linalg.norm(rf)
    # sp-DBA at threshold zero is the dense half trajectory bit for bit
    S = o.step(_inst(o, opc, (1, n, n), blk, 0.0, o.FLAG_PIN_K0 | o.FLAG_HALF), half0, steps, masks=True)
    assert S["masks"].all() and np.array_equal(S["state"], H)


def test_half_energy_and_mass_match_the_full_layout(oracle_mod):
    o = oracle_mod
    n = 16
    c = inputs.uniform_field(1002, 3, (n, n, n), 0.1, 0.02)
    ef, mf = o.ch_energy(_inst(o, o.OP_CH, (n, n, n), (4, 4, 4), 0.0, o.FLAG_PIN_K0), np.fft.fftn(c).ravel())
    eh, mh = o.ch_energy(_inst(o, o.OP_CH, (n, n, n), (4, 4, 4), 0.0, o.FLAG_HALF), o.rfft(c).ravel())
    assert abs(eh - ef) <= 1e-12 * abs(ef) and abs(mh - mf) <= 1e-14
    # a gradient-only check: a single cosine mode, closed form
    x = np.arange(n)
    cc = 0.3 * np.cos(2 * np.pi * 3 * x / n)[None, None, :] * np.ones((n, n, 1))
    e1, _ = o.ch_energy(_inst(o, o.OP_CH, (n, n, n), (4, 4, 4), 0.0, o.FLAG_HALF), o.rfft(cc).ravel())
    bulk = np.sum(0.25 * (cc ** 2 - 1) ** 2)
    k2 = (2 * np.pi * 3 / n) ** 2
    grad = 0.5 * 1.0 * k2 * np.sum(0.5 * 0.3 ** 2 * np.ones(n ** 3))  # (kappa/2) sum |grad c|^2
    assert abs(e1 - (bulk + grad)) <= 1e-11 * abs(bulk + grad)


def test_half_sp_dba_conserves_mass_and_freezes_blocks(oracle_mod):
    o = oracle_mod
    n = 32
    c0 = inputs.uniform_field(1001, 9, (n, n), 0.0, 0.05)
    inst = _inst(o, o.OP_CH, (1, n, n), (1, 8, 8), 3e-2, o.FLAG_PIN_K0 | o.FLAG_HALF)
    h0 = o.rfft(c0).ravel()
    res = o.step(inst, h0, 30, masks=True)
    assert res["state"][0] == h0[0]  # k = 0: s = 0, a = 1, exact
    per_step = res["masks"].reshape(30, -1).sum(axis=1)
    assert per_step.min() < inst.n_blocks and res["masks"][:, 0, 0].all()


def test_half_layout_rejects_complex_fields_and_bad_blocks(oracle_mod):
    o = oracle_mod
    q = np.zeros(16 * 9, np.complex128)
    bad = [o.Inst(op=o.OP_NLSE, dims=(1, 1, 16), block=(1, 1, 4), tau=0.1, dx=1.0, dt=0.1,
                  p=(-21.7, 1.3, 0.0), flags=o.FLAG_HALF),
           _inst(o, o.OP_CH, (1, 16, 16), (1, 4, 16), 0.1, o.FLAG_HALF),  # x block does not divide nx/2
           _inst(o, o.OP_CH, (1, 16, 16), (1, 4, 1), 0.1, o.FLAG_HALF | o.FLAG_TRANSITION)]  # X_0 needs columns 0, 1
    for inst in bad:
        with pytest.raises(o.OracleError):
            o.apply(inst, q, q)


# ---------------------------------------------------------------------------
# transition states on the half layout (Supplementary S1.1 with the
# conjugate neighbour remap of S1.2)
# ---------------------------------------------------------------------------
N2, B2 = 32, 4
NBY, NBXM = N2 // B2, (N2 // 2) // B2


def _tr_inst(o, tau=1e-3, extra=0):
    return _inst(o, o.OP_CH, (1, N2, N2), (1, B2, B2), tau,
                 o.FLAG_HALF | o.FLAG_STATE | o.FLAG_TRANSITION | extra)


def _blk(by, bx):
    """Stored block id: columns below nx/2 first, then the column nx/2 (bx = NBXM)."""
    return NBY * NBXM + by if bx == NBXM else by * NBXM + bx


def _one_mode_in(cells):
    q = np.zeros((N2, N2 // 2 + 1), np.complex128)
    for by, bx in cells:
        q[by * B2 + 1, N2 // 2 if bx == NBXM else bx * B2 + 1] = 1.0
    return q.ravel()


def _states(o, cells, tau=1e-3):
    q = _one_mode_in(cells)
    m = o.apply(_tr_inst(o, tau), q, np.zeros_like(q))["mask"]
    return {int(b): int(v) for b, v in enumerate(m) if v}


@pytest.mark.parametrize("active,transition", [
    # a block of X_0 away from kx = 0's partners: its y and x neighbours, and
    # across kx = 0 the blocks of X_0 holding the mirrored rows -y (rows 8..11
    # mirror to 21..24: blocks 5 and 6)
    ((2, 0), [(1, 0), (3, 0), (2, 1), (5, 0), (6, 0)]),
    # row block 0 mirrors to rows 0 and 29..31: itself and block 7
    ((0, 0), [(1, 0), (7, 0), (0, 1)]),
    # the last block below nx/2: X_N at its own rows and at the mirrored ones
    # (rows 12..15 mirror to 17..20: blocks 4 and 5)
    ((3, NBXM - 1), [(2, NBXM - 1), (4, NBXM - 1), (3, NBXM - 2), (3, NBXM), (4, NBXM), (5, NBXM)]),
    # the column nx/2: beyond it the mirrored rows of X_{nbxm-1}
    ((2, NBXM), [(1, NBXM), (3, NBXM), (2, NBXM - 1), (5, NBXM - 1), (6, NBXM - 1)]),
])
def test_half_transition_states_hand_cases(oracle_mod, active, transition):
    o = oracle_mod
    got = _states(o, [active])
    want = {_blk(*active): 1}
    want.update({_blk(*c): 2 for c in transition})
    assert got == want


def test_half_transition_relation_is_symmetric(oracle_mod):
    """Conjugation is an involution, so if one active block turns a block
    into a transition block, that block, active alone, turns the first one
    into a transition block as well."""
    o = oracle_mod
    cells = [(by, bx) for by in range(NBY) for bx in range(NBXM + 1)]
    near = {_blk(*c): {b for b, v in _states(o, [c]).items() if v == 2} for c in cells}
    pairs = 0
    for a, nb in near.items():
        for b in nb:
            assert a in near[b], (a, b)
            pairs += 1
    assert pairs > 4 * len(cells)


def test_half_transition_weights_are_the_roll_off_of_the_frozen_faces(oracle_mod):
    """Active block (2, X_0): the transition block (1, X_0) borders the frozen
    block (0, X_0) on its low y face and the frozen block (1, X_1) on its high
    x face; across kx = 0 it meets the transition block (6, X_0) and on its
    high y face the active block.  Its weight is w(ly) w(B - 1 - lx) with
    w(i) = (1 - cos(pi i / (B - 1))) / 2."""
    o = oracle_mod
    rng = inputs.rng_for(83, 1)
    q = _one_mode_in([(2, 0)]) * 1e3
    shape = (N2, N2 // 2 + 1)
    q = q + 1e-6 * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).ravel()
    rhs = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).ravel()
    inst = _tr_inst(o, tau=1e-2)
    res = o.apply(inst, q, rhs)
    assert res["mask"][_blk(1, 0)] == 2 and res["mask"][_blk(1, 1)] == 0 and res["mask"][_blk(0, 0)] == 0
    cand = o.apply(_inst(o, o.OP_CH, (1, N2, N2), (1, B2, B2), 0.0, o.FLAG_HALF | o.FLAG_DENSE), q, rhs)["q"]
    w = 0.5 * (1.0 - np.cos(np.pi * np.arange(B2) / (B2 - 1)))
    got = res["q"].reshape(shape)
    c, q0 = cand.reshape(shape), q.reshape(shape)
    for ly in range(B2):
        for lx in range(B2):
            y, x = 1 * B2 + ly, lx
            sig = w[ly] * w[B2 - 1 - lx]
            assert abs(got[y, x] - (q0[y, x] + sig * (c[y, x] - q0[y, x]))) <= 1e-12 * abs(c[y, x] - q0[y, x]) + 1e-300


def test_half_transition_keeps_mass_and_threshold_zero_is_dense(oracle_mod):
    o = oracle_mod
    c0 = inputs.uniform_field(1001, 11, (N2, N2), 0.0, 0.05)
    h0 = o.rfft(c0).ravel()
    res = o.step(_tr_inst(o, tau=3e-2, extra=o.FLAG_PIN_K0), h0, 20, masks=True)
    assert res["state"][0] == h0[0]
    assert (res["masks"] == 2).any() and (res["masks"] == 0).any()
    dense = o.step(_inst(o, o.OP_CH, (1, N2, N2), (1, B2, B2), 0.0, o.FLAG_HALF | o.FLAG_DENSE), h0, 20)["state"]
    zero = o.step(_tr_inst(o, tau=0.0), h0, 20)["state"]
    assert np.array_equal(zero, dense)
