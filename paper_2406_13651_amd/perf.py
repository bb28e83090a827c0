"""Algorithmic HBM bytes of each kernel stage per launch.

Each stream a stage must read or write is counted once (no re-reads, no
cache effects); these are the byte counts the roofline figures divide by a
measured launch duration.  Sizes: complex64 = 8 bytes, float32 = 4 bytes.
"""


def stage_bytes(nx, ny, nz, looks, P, B, n_agents, K=0, fused=False):
    """Bytes per launch of each timing stage of one CLAMP iteration (K > 0:
    the 3D operator with K range frequencies, adding the two range passes and
    keeping the residual on the K x P cylinder; fused: the Mann step inside
    the update pass, whose own launch is then only the final reduction)."""
    L = looks
    n = nx * ny * nz
    band = 8 * ny * B          # one slice's band rows (complex64)
    extra = {}
    if K > 0:
        extra = {
            # box [K][P] in, every slice [nz][P] out
            "range_inv": L * 8 * P * (K + nz),
            # every slice in, box out
            "range_fwd": L * 8 * P * (nz + K),
        }
    out = {
        # resid (compact) in, band rows out
        "col_inv": L * nz * (8 * P + band),
        # band rows in, mu and the anchor in, band rows out
        "row_grad": L * nz * (band + ny * nx * (8 + 4) + band),
        # band rows in, D(a) F d (compact) out
        "col_fwd": L * nz * (band + 8 * P),
        # band rows, mu, anchor and w in; mu and r out
        "row_update": L * nz * (band + ny * nx * (8 + 4 + 4 + 8 + 4)),
        # resid and D(a) F d in, resid out
        "resid_update": L * (K if K > 0 else nz) * P * 24,
        # one pass over the volume: float32 in and out
        "prior_gauss": n * 8,
        # every agent's w and r in, w out, and w_bar out
        "mace_step": n * (12 * n_agents + 4),
    }
    if fused:
        del out["row_update"], out["mace_step"]
        # band rows, mu, anchor and u in, mu, r and u out per look; per voxel
        # x_bar and w_bar in and out, and with a prior its output in and its w
        # in and out
        prior = 12 if n_agents == looks + 1 else 0
        out["row_update_mann"] = L * nz * (band + ny * nx * (8 + 4 + 4 + 8 + 4 + 4)) + n * (16 + prior)
    out.update(extra)
    return out


def agent_bytes_min(nx, ny, nz, looks, P):
    """Lower bound for one forward-agent application with the gamma barrier:
    mu in and out, anchor in, r out, w in, the residual on the pupil in and out,
    d across the barrier, and D(a) F d across the barrier (48 + 32 alpha bytes
    per voxel-look)."""
    n = nx * ny * nz
    return looks * (48 * n + 32 * nz * P)
