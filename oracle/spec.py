"""Build an oracle Problem from a plain problem spec (oracle, test infrastructure only).

A spec is a dict of NumPy arrays and tuples (the seeded workloads produce them):
order, blocks [X1, X2, rho, C10, bc = 4 x (kind, g, time_fn, time_params, U),
forcing], interfaces, interface_data, dissipation, sources, receivers.  Time functions: 0 zero, 1 one,
2 cos(p0 t + p1), 3 Ricker(peak p0, centre p1) (Sec. 7.4).
"""
import numpy as np

from . import elastic as E, material as M, sources as Src


def tfun(kind, p):
    p = (0.0, 0.0) if p is None else tuple(p) + (0.0,) * (2 - len(p))
    if kind == 0:
        return lambda t: 0.0
    if kind == 1:
        return lambda t: 1.0
    if kind == 2:
        return lambda t: np.cos(p[0] * t + p[1])
    if kind == 3:
        return lambda t: Src.ricker(t, p[0], p[1])
    raise ValueError(kind)


def build(spec, beta=1.0):
    blocks = []
    for b in spec['blocks']:
        blocks.append(E.Block(b['X1'], b['X2'], b['rho'], M.full_from_c10(b['C10']),
                              order=spec['order'], beta=beta, operator=spec.get('operator', 'narrow')))
    itfs = [E.Interface(a, fa, bb, fb, reversed=bool(rev)) for (a, fa, bb, fb, rev) in spec.get('interfaces', [])]
    # jump data (Sec. 6): (interface index, V, Theta, time_fn, params), side a's order
    for (k, V, Th, tk, tp) in spec.get('interface_data', []):
        itfs[k].V = None if V is None else np.asarray(V, dtype=float)
        itfs[k].Theta = None if Th is None else np.asarray(Th, dtype=float)
        itfs[k].tfun = tfun(tk, tp)
    P = E.Problem(blocks, itfs, beta=beta)
    for k, b in enumerate(spec['blocks']):
        for f, (kind, g, tk, tp, U) in enumerate(b['bc']):
            if blocks[k].bc[f]['kind'] == E.INTERFACE:
                continue
            P.set_bc(k, f, kind, g=g, tfun=tfun(tk, tp) if g is not None else None, U=U)
        if b.get('forcing') is not None:
            F, tk, tp = b['forcing']
            P.forcing[k] = (F, tfun(tk, tp))
    # dissipative Robin terms V u_t (the remark after eq. sat_traction): (block, face, V [2][2][nf])
    for (k, f, V) in spec.get('dissipation', []):
        P.blocks[k].bc[f]['V'] = np.asarray(V, dtype=float)
    for (bid, x1, x2, f1, f2, amp, fp, t0) in spec.get('sources', []):
        P.sources.append(Src.point_source(bid, blocks[bid], x1, x2, (f1, f2), amp, fp, t0))
    return P


def receivers(spec, us):
    out = []
    for (bid, x1, x2) in spec.get('receivers', []):
        for a, b in zip(x1, x2):
            out.append(Src.sample(us[bid], a, b))
    return np.array(out)
