"""Cold / seeded / refresh schedule for a sequence of SCF steps.

The paper's schedule (section 2, paragraph "Eigenvectors evolution"): a few
standard iterations with the full direct solver first, then fast iterations
whose iterative solver is initialised with the previous eigenvectors, until
progress towards convergence flattens out; then a full iteration refreshes
the process and a new series of fast iterations follows.

The eigensolver cannot see SCF convergence itself, so the policy reads
"progress flattens" from what each seeded solve reports:

* how far the eigenvectors moved (``seed_sin_rms``, the RMS sine of the
  principal angles between the seed and the result; the paper observes the
  deviation angles decreasing monotonically once the SCF settles), and
* what the fast solve cost (filter column-degrees, ``col_degrees``).

A series is refreshed (next step cold) when the subspace moved more than
``max_sin_rms``, when the angles stopped shrinking for ``flat_steps``
consecutive steps (each at least ``flat_ratio`` times the previous one), or
when a seeded solve cost more than ``max_cost_growth`` times the cheapest
one of its series.  Angles below ``settled_sin_rms`` count as settled, not
flat: a sequence whose eigenvectors no longer move measurably has converged
as far as the eigensolver can tell, and refreshing it would only cost a
cold solve.  Host logic only: decisions come from the info
dictionaries ``gevp.Handle.solve`` returns with ``seed_monitor`` enabled.
"""
from dataclasses import dataclass, field
from typing import List


@dataclass
class RestartPolicy:
    direct_steps: int = 1
    max_sin_rms: float = 0.3
    flat_ratio: float = 0.95
    flat_steps: int = 2
    max_cost_growth: float = 2.0
    settled_sin_rms: float = 1e-10
    history: List[dict] = field(default_factory=list)

    def next_mode(self) -> str:
        """'cold' or 'seeded' for the next SCF step."""
        k = len(self.history)
        if k < self.direct_steps:
            return "cold"
        last = self.history[-1]
        if last["mode"] == "cold":
            return "seeded"
        series = self._series()
        sin = [h["sin_rms"] for h in series]
        if sin[-1] > self.max_sin_rms:
            return "cold"
        if len(sin) > self.flat_steps and sin[-1] > self.settled_sin_rms:
            tail = sin[-(self.flat_steps + 1):]
            if all(tail[i + 1] >= self.flat_ratio * tail[i] for i in range(self.flat_steps)):
                return "cold"
        costs = [h["cost"] for h in series]
        if costs[-1] > self.max_cost_growth * min(costs):
            return "cold"
        return "seeded"

    def record(self, mode: str, info: dict) -> None:
        """Record the solve just done (``mode`` as returned by next_mode)."""
        sin = info.get("seed_sin_rms", -1.0)
        if mode == "seeded" and sin < 0:
            raise ValueError("a seeded step needs the seed monitor (opts seed_monitor=True)")
        self.history.append({"mode": mode, "sin_rms": sin, "cost": int(info.get("col_degrees", 0)),
                             "outer_iters": int(info.get("outer_iters", 0))})

    def _series(self):
        """Seeded steps since the last cold one."""
        out = []
        for h in reversed(self.history):
            if h["mode"] == "cold":
                break
            out.append(h)
        return out[::-1]
