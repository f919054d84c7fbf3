"""CPU oracle for the PFB packet order and the averaged output -- TEST
INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module.  It shares no code with the GPU library.

What it defines (Ord et al., "The Murchison Widefield Array Correlator"):

- Appendix A, data format: a PFB lane carries 384 fine channels of the 64
  inputs of one PFB, packetised in f1 t [f2 a] order: the packet of channel
  group f1 and time t holds, fastest first, the inputs a in the PFB's order
  0, 16, 32, 48, 1, 17, ... (position k carries input 16 (k mod 4) + k div 4)
  and then the four fine channels f2 = f1 .. f1+3.  The groups f1 of fibre 0
  are 0, 4, 8, 12, 128, 132, ..., 2944, ..., 2956; fibre n adds 16 n.
- Appendix B: the XMAC server strips the headers and concatenates the four
  PFBs' packets, keeping each packet's input order: 4 x 64 = 256 inputs.
- Appendix C, GPU input/output: the XMAC correlates in that (packet) order and
  the products are remapped afterwards to the order the PFB inputs were
  presented in, conjugating those whose two inputs swap order.
- Sec. 3.4.3: the archived products may be averaged by two in time and in
  frequency.

Lane payload layout used here (headers, counters and checksums removed):
packet (c, s, t) of a lane for coarse channel c, group s = 0..3 and time t is
256 bytes at offset ((c * 4 + s) * T + t) * 256; byte 64 f2 + k is fine
channel f2 of packet position k.  The fine channel is 128 c + 16 n + 4 s + f2
for fibre n.
"""

from __future__ import annotations

import numpy as np


def pfb_input_at_position(k: int) -> int:
    """PFB input carried at packet position k (0..63), Appendix A."""
    return 16 * (k % 4) + k // 4


def pfb_antenna_order() -> list[int]:
    """The 64 PFB inputs in packet order."""
    return [pfb_input_at_position(k) for k in range(64)]


def fibre_channel_groups(fibre: int) -> list[int]:
    """First fine channel f1 of each of the 96 packet groups of a fibre, in
    stream order (Appendix A): four groups of four channels from each of the
    24 coarse channels of 128."""
    return [128 * (g // 4) + 4 * (g % 4) + 16 * fibre for g in range(96)]


def ingest(lanes: list[np.ndarray], n_pfb: int, n_coarse: int, n_time: int, natural: bool) -> np.ndarray:
    """Assemble the (time, channel, input) buffer from 8 * n_pfb lane payloads
    (lane of PFB b, fibre n at index 8 b + n).  Input index 64 b + k keeps the
    packet position (the paper's XMAC order); natural=True puts the sample at
    64 b + (PFB input of position k)."""
    n_chan, n_inputs = 128 * n_coarse, 64 * n_pfb
    out = np.zeros((n_time, n_chan, n_inputs), dtype=np.uint8)
    for b in range(n_pfb):
        for n in range(8):
            pay = np.asarray(lanes[8 * b + n], dtype=np.uint8).reshape(n_coarse, 4, n_time, 4, 64)
            for c in range(n_coarse):
                for s in range(4):
                    for f2 in range(4):
                        f = 128 * c + 16 * n + 4 * s + f2
                        for k in range(64):
                            col = 64 * b + (pfb_input_at_position(k) if natural else k)
                            out[:, f, col] = pay[c, s, :, f2, k]
    return out.reshape(-1)


def packet_index(i: int) -> int:
    """Packet-order input index of natural input i (inverse of the PFB map
    inside each block of 64)."""
    b, a = divmod(i, 64)
    for k in range(64):
        if pfb_input_at_position(k) == a:
            return 64 * b + k
    raise ValueError(i)


def remap(vis_pkt: np.ndarray, n_inputs: int) -> np.ndarray:
    """Natural-order lower triangle from the packet-order one:
    V[i][j] = V_pkt[P(i)][P(j)] if P(i) >= P(j), else conj(V_pkt[P(j)][P(i)]).
    vis_pkt: (F, B, 2) with b = i (i + 1) / 2 + j."""
    vis_pkt = np.asarray(vis_pkt)
    out = np.empty_like(vis_pkt)
    P = [packet_index(i) for i in range(n_inputs)]
    for i in range(n_inputs):
        for j in range(i + 1):
            pi, pj = P[i], P[j]
            b = i * (i + 1) // 2 + j
            if pi >= pj:
                out[:, b, :] = vis_pkt[:, pi * (pi + 1) // 2 + pj, :]
            else:
                src = vis_pkt[:, pj * (pj + 1) // 2 + pi, :]
                out[:, b, 0] = src[:, 0]
                out[:, b, 1] = -src[:, 1]
    return out


def channel_sum(vis: np.ndarray, f_avg: int) -> np.ndarray:
    """Sum of f_avg adjacent channels: out[g] = sum_q vis[g f_avg + q] (int64)."""
    vis = np.asarray(vis, dtype=np.int64)
    F = vis.shape[0]
    assert F % f_avg == 0
    out = np.zeros((F // f_avg,) + vis.shape[1:], dtype=np.int64)
    for g in range(F // f_avg):
        for q in range(f_avg):
            out[g] += vis[g * f_avg + q]
    return out
