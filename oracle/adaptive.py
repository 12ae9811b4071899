"""The fine-level adaptive correction of the paper's preconditioner (test
infrastructure only: see the package header).

Tab. solver-config: after the multigrid cycle, an additional correction on the
finest level, 20 steps of an inner FGMRES iteration with restart 20,
preconditioned by the 3x3 node-block Jacobi operator, applied only if it
reduces the residual norm.  With z = V(v) the cycle's output and s = v - K z,
the inner iteration solves K d = s from d = 0; z + d replaces z when
||v - K (z + d)|| < ||v - K z||.  The preconditioner so obtained depends on
its argument nonlinearly, which is why the outer method must be flexible
(Sec. 3.5).
"""
import numpy as np

from . import fgmres as fg
from . import multigrid as mg


def adaptive_preconditioner(levels, inner_steps=20):
    """v -> z: one V-cycle followed by the accepted-or-rejected fine-level
    correction.  The returned callable keeps one keep/reject flag per call in
    its attribute ``log``."""
    K = levels[0].K
    Binv = levels[0].Binv
    log = []

    def M(v):
        z = mg.vcycle(levels, v)
        if inner_steps <= 0:
            log.append(False)
            return z
        s = v - K @ z
        r0 = np.linalg.norm(s)
        inner = fg.fgmres(lambda y: K @ y, lambda y: Binv @ y, s, restart=inner_steps, max_iters=inner_steps,
                          tol=0.0)
        r1 = np.linalg.norm(s - K @ inner.x)
        ok = bool(r1 < r0)
        log.append(ok)
        return z + inner.x if ok else z

    M.log = log
    return M
