"""Small hand-built cases for the tests (inputs only, no solver arithmetic)."""
import math

import numpy as np

from paper_2310_06650_amd.synth import GridCase


def tiny_case(n_bus, br_from, br_to, br_x, gen_bus, T=3, br_r=None, ctg=None,
              dt=None, seg_size=None, seg_cost=None, **over):
    L = len(br_from)
    G = len(gen_bus)
    br_x = np.asarray(br_x, dtype=float)
    br_r = np.zeros(L) if br_r is None else np.asarray(br_r, dtype=float)
    seg_size = (np.full((G, 3), 1.0) if seg_size is None
                else np.asarray(seg_size, dtype=float))
    seg_cost = (np.tile([10.0, 20.0, 30.0], (G, 1)) if seg_cost is None
                else np.asarray(seg_cost, dtype=float))
    pmax = seg_size.sum(axis=1)
    kw = dict(
        n_bus=n_bus, n_branch=L, n_gen=G, n_period=T, n_seg=seg_size.shape[1],
        br_from=np.asarray(br_from, dtype=np.int32),
        br_to=np.asarray(br_to, dtype=np.int32), br_r=br_r, br_x=br_x,
        br_bch=np.zeros(L), br_smax=np.full(L, 1.0), br_smax_ctg=np.full(L, 1.2),
        gen_bus=np.asarray(gen_bus, dtype=np.int32), gen_pmin=0.1 * pmax,
        gen_pmax=pmax, gen_qmin=-0.3 * pmax, gen_qmax=0.5 * pmax,
        gen_rmax=0.1 * pmax, gen_ru=0.5 * pmax, gen_rd=0.5 * pmax,
        gen_ru_su=0.4 * pmax, gen_rd_sd=0.4 * pmax, gen_p0=0.5 * pmax,
        gen_u0=np.ones(G), gen_c_on=np.ones(G), gen_c_su=np.full(G, 10.0),
        gen_c_sd=np.full(G, 1.0), gen_c_r=np.ones(G), gen_seg_cost=seg_cost,
        gen_seg_size=seg_size, load_p=np.full((T, n_bus), 0.2),
        load_q=np.full((T, n_bus), 0.05), reserve_req=np.full(T, 0.1),
        dt=np.ones(T) if dt is None else np.asarray(dt, dtype=float),
        v_min=np.full(n_bus, 0.9), v_max=np.full(n_bus, 1.1), c_p=100.0,
        c_q=100.0, c_s=50.0, c_ang=50.0, ang_max=72.0 * math.pi / 180.0,
        c_rsv=20.0, rho=30.0, load_value=60.0,
        ctg_list=np.asarray([] if ctg is None else ctg, dtype=np.int32))
    kw.update(over)
    return GridCase(**kw)
