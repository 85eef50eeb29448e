"""Plain evaluation of the CREDIT profitability model (Sec. III-B to III-D).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function is one
equation of the paper written out in FP64 Python, in the paper's notation, with
no fitting and no shortcuts:

* ``capacity_legal``      Eq. (3)  staging capacity
* ``hbm_traffic``         Eq. (4)  per-row HBM bytes, baseline vs staged
* ``protocol_cost``       Eq. (6)  replicated push/all-gather bytes and barriers
* ``effective_bandwidth`` / ``t_save``  Eq. (7)
* ``waves`` / ``t_replay`` / ``t_dsm``  Eq. (8)
* ``t_deposit``           the non-overlapped deposit residual [T_w - T_input]^+
* ``delta_t``             Eq. (9)
* ``crossover_width``     N*, the smallest tested width with a profitable legal P
* ``structural_screen``   the rules that reject a pattern before any timing
                          (elementwise and scalar-output reductions, scans,
                          selection / stencil kernels)

``Workload`` is the static description the model consumes (b_B, b_keep,
b_reread, q_l, L), derived here from a stage structure: which input tensors each
reduction stage reads, which the final apply pass reads, and what it writes.  In
the global-reread schedule every stage and the apply pass stream their inputs
from HBM; in the staged schedule every input is read once.

The MI355X adaptation used by the product's analytic selector differs only in
what S, P and the exchange mean (k co-resident workgroups exchanging through the
L2 instead of P CTAs of a cluster); ``amd_delta_t`` writes that form out.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Sequence


@dataclass(frozen=True)
class Workload:
    """Stage structure of a reduction-reuse kernel (Eq. (1)).

    inputs:  bytes per element of each input tensor, by name
    stages:  for each stage l, (names of inputs it reads, q_l)
    apply:   names of inputs the output pass reads
    outputs: bytes per element written
    """

    inputs: Dict[str, float]
    stages: List[tuple]
    apply: Sequence[str]
    outputs: float
    keep: Sequence[str] = field(default=())

    @property
    def L(self) -> int:
        return len(self.stages)

    @property
    def q(self) -> List[int]:
        return [qs for _, qs in self.stages]

    def b_B(self) -> float:
        """Baseline (global-reread) bytes per element, output included."""
        b = sum(sum(self.inputs[n] for n in reads) for reads, _ in self.stages)
        b += sum(self.inputs[n] for n in self.apply)
        return b + self.outputs

    def b_cluster(self) -> float:
        """Staged schedule: every input once, plus the output."""
        return sum(self.inputs.values()) + self.outputs

    def b_reread(self) -> float:
        return self.b_B() - self.b_cluster()

    def b_keep(self) -> float:
        names = self.keep if self.keep else tuple(self.inputs)
        return sum(self.inputs[n] for n in names)


def hbm_traffic(w: Workload, N: int, D_fixed_per_elem: float | None = None):
    """Eq. (4): (D_base, D_cluster) per row.  D_fixed is the traffic common to
    both schedules; here every input once plus the output."""
    fixed = w.b_cluster() if D_fixed_per_elem is None else D_fixed_per_elem
    D_fixed = N * fixed
    return D_fixed + N * w.b_reread(), D_fixed


def capacity_legal(N: int, P: int, b_keep: float, S_scratch: float, S_max: float) -> bool:
    """Eq. (3): ceil(N/P) * b_keep + S_scratch <= S_max."""
    return math.ceil(N / P) * b_keep + S_scratch <= S_max


def protocol_cost(P: int, q: Sequence[int], s: float):
    """Eq. (6): remote write bytes, remote read bytes, barriers per row."""
    return s * P * (P - 1) * sum(q), 0.0, 2 * len(q)


def effective_bandwidth(M: int, N: int, b_B: float, T_B: float) -> float:
    """Eq. (7), first line."""
    return M * N * b_B / T_B


def t_save(M: int, N: int, b_reread: float, B_eff: float) -> float:
    """Eq. (7), second line: time to stream the eliminated reread."""
    return M * N * b_reread / B_eff


def waves(M: int, S: int, P: int) -> int:
    """Eq. (8): W = ceil(M / floor(S / P))."""
    return math.ceil(M / (S // P))


def t_replay(M: int, N: int, P: int, S: int, b_keep: float, f: float, B_smem_r: float) -> float:
    """Eq. (8): W * ceil(N/P) * b_keep / (f * B_SMEM^r)."""
    return waves(M, S, P) * math.ceil(N / P) * b_keep / (f * B_smem_r)


def t_dsm(M: int, P: int, S: int, q: Sequence[int], s: float, f: float, B_dsm_w: float) -> float:
    """Eq. (8): s * W * (P - 1) * sum q / (f * B_DSM^w(P)); not multiplied by P."""
    return s * waves(M, S, P) * (P - 1) * sum(q) / (f * B_dsm_w)


def t_deposit(T_smem_w: float, T_input: float) -> float:
    """[T_SMEM^w - T_input]^+ (the deposit residual not hidden by the load)."""
    return max(T_smem_w - T_input, 0.0)


def delta_t(T_save: float, T_ctrl: float, T_replay: float, T_deposit: float, T_dsm: float) -> float:
    """Eq. (9)."""
    return T_save - T_ctrl - T_replay - T_deposit - T_dsm


def crossover_width(widths: Sequence[int], legal_and_profitable) -> int | None:
    """N*: smallest tested width for which some legal P has Delta T > 0.
    `legal_and_profitable(N)` returns True when that holds."""
    for N in sorted(widths):
        if legal_and_profitable(N):
            return N
    return None


def structural_screen(w: Workload, barriers_per_row=None, remote_state_per_row=None,
                      widths: Sequence[int] = (4096, 65536)) -> List[str]:
    """The model's structural rejection rules (end of Sec. III-D, and the
    negative controls of Sec. IV-D): a pattern is outside the reduction-reuse
    class, whatever its width, when

    * it rereads nothing (b_reread = 0: elementwise maps, reductions with a
      scalar output), so there is no source time to recover;
    * its synchronisation count per row K grows with N (scans: an ordered
      carry crosses every slice), so widening adds cost faster than it can
      be amortised;
    * the state exchanged per row grows with N (selection, stencils: halos or
      candidate lists instead of sum q_l compact scalars).

    barriers_per_row(N) and remote_state_per_row(N) default to the paper's
    protocol, K = 2L and sum q_l, which do not depend on N.  Returns the
    reasons for rejection; an empty list means the pattern is in the class."""
    K = barriers_per_row or (lambda N: 2 * w.L)
    R = remote_state_per_row or (lambda N: sum(w.q))
    lo, hi = min(widths), max(widths)
    reasons = []
    if w.b_reread() <= 0.0:
        reasons.append("no reread to recover")
    if K(hi) > K(lo):
        reasons.append("synchronisation grows with N")
    if R(hi) > R(lo):
        reasons.append("exchanged state grows with N")
    return reasons


# ------------------------------------------------------------------ MI355X form
def amd_waves(M: int, S: int, o: int, k: int) -> int:
    """Row-group waves when o workgroups fit per CU and a row uses k of them:
    W = ceil(M / floor(S * o / k))."""
    return math.ceil(M / max(1, (S * o) // k))


def amd_delta_t(*, M: int, N: int, k: int, S: int, o: int, f: float, b_B: float,
                b_reread: float, T_B: float, T_ctrl: float, lds_bytes_per_wg: float,
                B_lds_r: float, s: float, q: Sequence[int], B_x_w: float) -> float:
    """Eq. (9) with the MI355X terms: T_save from the achieved baseline rate
    (Eq. (7)); T_replay charged only for the LDS-held part of a slice (the
    register-held part is replayed for free); T_xchg the time to write one
    slot per statistic per peer-visible partial, W (k - 1) sum q s / (f B_x^w);
    T_deposit = 0 (the deposit is the load's own register write)."""
    W = amd_waves(M, S, o, k)
    ts = T_B * b_reread / b_B
    tr = W * lds_bytes_per_wg / (f * B_lds_r) if lds_bytes_per_wg > 0 else 0.0
    tx = s * W * (k - 1) * sum(q) / (f * B_x_w)
    return delta_t(ts, T_ctrl, tr, 0.0, tx)


# ------------------------------------------------------------------ workloads
def paper_workloads() -> Dict[str, Workload]:
    """Stage structures of five of the paper's FP32 workloads (Sec. IV-A),
    as read from their definitions.  Used to reproduce the printed traffic."""
    f = 4.0
    return {
        # LayerNorm backward, statistics recomputed: (mean, var) from x, then
        # (sum g, sum g*xhat) from x and dy, then dx from x and dy.
        "layernorm_bwd": Workload({"x": f, "dy": f}, [(("x",), 2), (("x", "dy"), 2)],
                                  ("x", "dy"), f),
        # Softmax-from-logits backward: max, sum exp, sum dy*y, then dx.
        "softmax_logits_bwd": Workload({"x": f, "dy": f},
                                       [(("x",), 1), (("x",), 1), (("x", "dy"), 1)],
                                       ("x", "dy"), f),
        # Pearson-correlation backward: the five moments of (x, y) in one
        # stage, then dx and dy.
        "pearson_bwd": Workload({"x": f, "y": f}, [(("x", "y"), 5)], ("x", "y"), 2 * f),
        # Row-wise int8 quantization: amax, then the int8 codes.
        "quant_int8": Workload({"x": f}, [(("x",), 1)], ("x",), 1.0),
        # Weighted-variance backward: (W, sum w x), then sum w (x - mu)^2, then
        # dx and dw each written by its own pass over (x, w).
        "wvar_bwd": Workload({"x": f, "w": f}, [(("x", "w"), 2), (("x", "w"), 1)], ("x", "w", "x", "w"), 2 * f),
    }


def credit_workloads(e: float) -> Dict[str, Workload]:
    """The build's operators with I/O element size e (bytes), global-reread
    schedule of the two-pass variant: one statistics pass, one apply pass."""
    return {
        "softmax_fwd": Workload({"x": e}, [(("x",), 2)], ("x",), e),
        "layernorm_fwd": Workload({"x": e}, [(("x",), 2)], ("x",), e),
        "rmsnorm_fwd": Workload({"x": e}, [(("x",), 1)], ("x",), e),
        "softmax_bwd": Workload({"y": e, "dy": e}, [(("y", "dy"), 1)], ("y", "dy"), e),
        "layernorm_bwd": Workload({"x": e, "dy": e}, [(("x", "dy"), 2)], ("x", "dy"), e),
        "rmsnorm_bwd": Workload({"x": e, "dy": e}, [(("x", "dy"), 1)], ("x", "dy"), e),
    }
