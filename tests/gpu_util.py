"""Helpers shared by the GPU tests: run the HIP path through the C-ABI and the
oracle on the same seeded inputs."""
import numpy as np

import paper_2402_03074_amd as H


def rel_linf(a, b):
    """max |a - b| / max |b| over one array."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_err(a, b, lead):
    """max over the leading `lead` indices (components, moment direction) of
    rel_linf of the remaining cell array."""
    a = np.asarray(a)
    b = np.asarray(b)
    return max(rel_linf(a[idx], b[idx]) for idx in np.ndindex(*a.shape[:lead]))


def state_err(P, got, ref, floor=0.0):
    """(error of the averages, error of the moments), per-array relative L-inf.
    floor > 0: a moment array is measured against at least `floor` times the
    largest cell average of its component (for moment arrays that are zero up
    to rounding, where max |ref| is itself rounding noise)."""
    eu = rel_err(got[0], ref[0], 1)
    if floor <= 0.0:
        return eu, rel_err(got[1], ref[1], 2)
    gm, rm = np.asarray(got[1]), np.asarray(ref[1])
    em = 0.0
    for d, k in np.ndindex(*rm.shape[:2]):
        den = max(np.abs(rm[d, k]).max(), floor * np.abs(ref[0][k]).max(), 1e-300)
        em = max(em, float(np.abs(gm[d, k] - rm[d, k]).max() / den))
    return eu, em


def to_gpu(x, dtype=None):
    import torch
    t = torch.tensor(np.ascontiguousarray(x), device="cuda")
    return t if dtype is None else t.to(dtype)


def solver_for(P, precision="fp64", **kw):
    """Single-instance GPU solver mirroring an oracle Problem."""
    bc = [{0: "periodic", 1: "transmissive", 2: "reflective"}[b] for b in P.bc]
    if P.dim == 1:
        inst = H.make_inst(P.nx, 1, P.domain[:2], bc)
    else:
        inst = H.make_inst(P.nx, P.ny, P.domain, bc)
    p = P.params
    weights = {0: "scale_invariant", 1: "zq", 2: "linear"}[p.weights]
    opts = dict(weights=weights, char_decomp=int(p.char_decomp), adv=(p.adv_x, p.adv_y),
                gas_gamma=p.gas_gamma, gamma_low=p.gamma_low, eps=p.eps)
    opts.update(kw)
    return H.Solver(P.dim, P.eq, [inst], precision=precision, **opts)


def flat(P, u, m):
    """Oracle layout -> C-ABI layout (cells flattened, x fastest)."""
    return u.reshape(P.ncomp, -1), m.reshape(P.dim, P.ncomp, -1)


def unflat(P, u, m):
    return u.reshape(P.shape), m.reshape((P.dim,) + P.shape)


def gpu_three_stages(S, P, u0, m0, dt, alpha, inputs=None):
    """Run stages 0, 1, 2 on the GPU.  inputs: optional list of the stage
    inputs (u, m) for stages 1 and 2 (taken from the oracle); otherwise the
    GPU's own outputs are chained.  Returns the three stage outputs (numpy,
    oracle layout)."""
    import torch
    mdt = S.mom_dtype
    uf, mf = flat(P, u0, m0)
    ug, mg = to_gpu(uf), to_gpu(mf, mdt)
    al = to_gpu(np.array([[alpha[0], alpha[1] if len(alpha) > 1 else 0.0]]))
    dtg = to_gpu(np.array([dt]))
    outs = []
    cur = (ug, mg)
    for s in range(3):
        if s > 0 and inputs is not None:
            ui, mi = flat(P, *inputs[s - 1])
            cur = (to_gpu(ui), to_gpu(mi, mdt))
        uo, mo = S.empty_state()
        S.stage(s, dtg, al, cur[0], cur[1], uo, mo)
        torch.cuda.synchronize()
        outs.append(unflat(P, uo.cpu().numpy(), mo.double().cpu().numpy()))
        if s == 0:
            keep0 = (ug, mg)  # the base must stay alive until stage 2
        cur = (uo, mo)
    del keep0
    return outs


def oracle_three_stages(P, u0, m0, dt, alpha):
    outs = []
    u, m, base = P.stage(0, dt, alpha, u0, m0)
    outs.append((u, m))
    u, m, _ = P.stage(1, dt, alpha, u, m, base)
    outs.append((u, m))
    u, m, _ = P.stage(2, dt, alpha, u, m, base)
    outs.append((u, m))
    return outs


def assert_mixed_stage_close(name, P, u0, dt, alpha, got, ref):
    """The mixed form's one-stage bar.  Averages: 2e-6 relative (FP32 fluxes
    times dt/dx).  Moments: 2e-5 of their maximum plus 1e-6 of the flux scale
    (dt/h)(1 + alpha) max|U|: they are formed in FP32 as v^ + dt F2, whose
    flux terms are of that size, so that rounding, not the moments' own size,
    sets the error where the moments are small (measured: at most 1.1e-7 of
    the flux scale, about two FP32 roundings)."""
    h = (P.dx,) if P.dim == 1 else (P.dx, P.dy)
    scale = (1.0 + max(alpha)) * max(np.abs(u0).max(), 1e-300)
    for s in range(3):
        eu, _ = state_err(P, got[s], ref[s])
        assert eu <= 2e-6, (name, s, eu)
        gm, rm = got[s][1], ref[s][1]
        worst = 0.0
        for d in range(P.dim):
            for k in range(P.ncomp):
                err = np.abs(gm[d, k] - rm[d, k]).max()
                worst = max(worst, err / (dt / h[d] * scale))
                assert err <= 2e-5 * np.abs(rm[d, k]).max() + 1e-6 * dt / h[d] * scale, \
                    (name, s, d, k, err)
        print(f"[gpu] mixed {name} stage {s}: averages {eu:.1e}, moments {worst:.1e} "
              f"of the flux scale", flush=True)
