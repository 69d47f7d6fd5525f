"""Error predictions of the GPU parity tests: the error model of oracle/precision.py (the
matrix-core rounding measured on gfx950 and the accumulation chains the context reports),
with the emulated rows Y = L^H A cached per case, since one case is usually checked against
several kernel configurations."""
from collections import OrderedDict

from oracle import precision as pr

_ROWS = OrderedDict()
_KEEP = 6


def predicted(key, m_blocks, L_list, w_q, mode, n_s, plan):
    """Emulated V(k) of the HERK form in ``mode`` for the blocks of one k. key names the
    blocks and factors (the cache key of their emulated rows); plan: the context's
    Exchange.accumulation_plan()."""
    if mode == "fp64":
        return pr.vx_k_emulated(m_blocks, L_list, w_q, mode, n_s)
    ns = [int(n_s)] * len(m_blocks) if isinstance(n_s, int) else [int(x) for x in n_s]
    rk = (key, mode)
    if rk not in _ROWS:
        _ROWS[rk] = pr.emulated_rows(m_blocks, L_list, mode, ns)
        while len(_ROWS) > _KEEP:
            _ROWS.popitem(last=False)
    _ROWS.move_to_end(rk)
    return pr.emulated_gram(_ROWS[rk], w_q, mode, ns, m_blocks[0].shape[0], plan)
