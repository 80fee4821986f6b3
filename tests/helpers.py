"""Shared test helpers: running the oracle and the HIP path on the same seeded
inputs and comparing what they produce."""
from __future__ import annotations

import numpy as np

E_COMPS = ("Ex", "Ey", "Ez")
B_COMPS = ("Bx", "By", "Bz")


def rel_l2(a_list, b_list):
    num = sum(float(np.sum((np.asarray(a) - np.asarray(b)) ** 2)) for a, b in zip(a_list, b_list))
    den = sum(float(np.sum(np.asarray(b) ** 2)) for b in b_list)
    return np.sqrt(num / den) if den > 0 else np.sqrt(num)


def oracle_sim(wl, laser=True, storage=64):
    """The oracle loaded with a workload: its explicit arrays, or its species
    description through the oracle's own loader (rounded to FP32 storage when
    storage == 32); its laser description or incident-field table."""
    import oracle
    s = oracle.Sim(wl["grid"])
    if "x" in wl:
        s.set_particles(wl["x"], wl["u"], wl["w"])
    else:
        s.particles_init(wl["species"])
        if storage == 32:
            s.round_storage()
    L = wl.get("laser")
    if laser and L:
        if "a0" in L:
            s.add_laser(L)
        else:
            s.set_laser(ey=L.get("ey"), ez=L.get("ez"))
    return s


def oracle_run(wl, nsteps, laser=True, storage=64):
    s = oracle_sim(wl, laser=laser, storage=storage)
    s.step(nsteps)
    return s


def gpu_sim(wl, precision, **kw):
    from paper_1511_03878_amd.sim import Sim
    return Sim.from_workload(wl, precision=precision, **kw)


def fields_of(sim, comps, oracle_layout=False):
    """Field components; the oracle's (fn_z, fn_y, fn_x) arrays of a 2-D box are
    reduced to (fn_y, fn_x) like the GPU's."""
    out = []
    for c in comps:
        f = sim.field(c)
        out.append(f[0] if oracle_layout and f.shape[0] == 1 else f)
    return out


def compare_fields(gpu, orc):
    """(rel-L2 of the E group, rel-L2 of the B group) between a GPU sim and an oracle sim."""
    e = rel_l2(fields_of(gpu, E_COMPS), fields_of(orc, E_COMPS, True))
    b = rel_l2(fields_of(gpu, B_COMPS), fields_of(orc, B_COMPS, True))
    return e, b


def neighbour_patch(p, code, np_, periodic):
    """Destination patch of direction code (dx+1) + 3 (dy+1) from patch p."""
    px, py = p % np_[0], p // np_[0]
    qx, qy = px + code % 3 - 1, py + code // 3 - 1
    if not (0 <= qx < np_[0]):
        if not periodic[0]:
            return -1
        qx %= np_[0]
    if not (0 <= qy < np_[1]):
        if not periodic[1]:
            return -1
        qy %= np_[1]
    return qx + np_[0] * qy


def neighbour_patch3(p, code, np_):
    """Destination patch of direction code (dx+1) + 3 (dy+1) + 9 (dz+1) from
    patch p of a periodic 3-D patch grid."""
    q = [p % np_[0], (p // np_[0]) % np_[1], p // (np_[0] * np_[1])]
    dd = [code % 3 - 1, (code // 3) % 3 - 1, code // 9 - 1]
    q = [(q[a] + dd[a]) % np_[a] for a in range(3)]
    return q[0] + np_[0] * (q[1] + np_[1] * q[2])
