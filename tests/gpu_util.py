"""Helpers shared by the GPU parity tests (host/device copies, pairing a HIP
hierarchy with an oracle hierarchy built from the same seeded inputs)."""
import numpy as np
import torch

from bf16_definition import bf16_nearest_even

ORACLE_KEYS = ("theta", "max_coarse", "max_levels", "smoother", "omega", "nu_pre", "nu_post", "symmetric")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def pair(rp, ci, v, **kw):
    """(HIP hierarchy, oracle hierarchy) for the same matrix and parameters."""
    import oracle
    from paper_2606_09001_amd.solver import AmgHierarchy
    print(f"[case] n={len(rp) - 1} nnz={len(ci)} params={kw}", flush=True)
    okw = {k: kw[k] for k in ORACLE_KEYS if k in kw}
    O = oracle.OracleHierarchy(rp, ci, v, **okw)
    H = AmgHierarchy(dev(rp), dev(ci), dev(v), **kw)
    return H, O


def assert_hierarchy_bitexact(H, O, mixed=False):
    st = H.stats()
    assert st["num_levels"] == O.num_levels, (st["num_levels"], O.num_levels)
    for l in range(O.num_levels):
        o = O.level(l)
        coarsest = l == O.num_levels - 1
        assert st["n"][l] == o["n"]
        names = ["A_rp", "A_ci", "A_v", "dinv", "sw"]
        if not coarsest:
            names += ["agg", "P_rp", "P_ci", "P_v", "R_rp", "R_ci", "R_v", "G_rp", "G_ci"]
            assert st["rho"][l] == o["rho"] and st["omega_p"][l] == o["omegaP"], l
        for name in names:
            g = host(H.export(l, name))
            ref = o[name]
            assert g.shape == ref.shape, (l, name, g.shape, ref.shape)
            if ref.dtype == np.float64:
                assert np.array_equal(g.view(np.int64), ref.view(np.int64)), (l, name)
            else:
                assert np.array_equal(g, ref), (l, name)
        if mixed:
            a32 = host(H.export(l, "A_v32"))
            assert np.array_equal(a32, o["A_v"].astype(np.float32)), (l, "A_v32")
            sw32 = host(H.export(l, "sw32"))
            assert np.array_equal(sw32.view(np.int32), o["sw"].astype(np.float32).view(np.int32)), (l, "sw32")
            if not coarsest:
                for name, src in (("P_bf16", "P_v"), ("R_bf16", "R_v")):
                    gb = host(H.export(l, name)).view(np.uint16).astype(np.int32)
                    f32 = torch.from_numpy(o[src].astype(np.float32))
                    ref = bf16_nearest_even(f32.view(torch.int32)).numpy()
                    assert np.array_equal(gb, ref), (l, name)
    # coarse factor: tolerance (different summation order)
    Lo = O.coarse_factor()
    nL = Lo.shape[0]
    m = int(round(np.sqrt(H.export(O.num_levels - 1, "coarse_factor").numel())))
    Lg = host(H.export(O.num_levels - 1, "coarse_factor")).reshape(m, m)[:nL, :nL]
    assert np.max(np.abs(Lg - Lo)) <= 1e-12 * np.abs(Lo).max()
    # explicit coarse inverse (stored transposed) against LAPACK's inverse of the
    # oracle's coarsest matrix; its FP32 copy is that inverse rounded to nearest
    o = O.level(O.num_levels - 1)
    Ac = np.zeros((nL, nL))
    rows = np.repeat(np.arange(nL), np.diff(o["A_rp"]))
    Ac[rows, o["A_ci"]] = o["A_v"]
    Ig = host(H.export(O.num_levels - 1, "coarse_inv")).reshape(m, m)
    Iref = np.linalg.inv(Ac)
    assert np.max(np.abs(Ig[:nL, :nL].T - Iref)) <= 1e-10 * np.abs(Iref).max()
    assert not Ig[nL:, :nL].any() and not Ig[:nL, nL:].any()
    if mixed:
        I32 = host(H.export(O.num_levels - 1, "coarse_inv32")).reshape(m, m)
        assert np.array_equal(I32.view(np.int32), Ig.astype(np.float32).view(np.int32)), "coarse_inv32"
