"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that the pins catch
each one: a pin set that a dropped term, flipped sign or shifted index survives would not pin
anything."""
import types

import numpy as np
import pytest

import oracle as O
from tests.test_oracle_pins import ALL_CHECKS


def _copy(**over):
    ns = types.SimpleNamespace(**{k: getattr(O, k) for k in dir(O) if not k.startswith("_")})
    for k, v in over.items():
        setattr(ns, k, v)
    # functions that call siblings must see the mutant, so rebind the composite ones
    if "search" not in over:
        def search(data, delays, widths, threshold, beam=0, nrep=None, t_offset=0):
            x = ns.dedisperse(data, delays)
            if nrep is None:
                nrep = x.shape[1] - max(widths) + 1
            return x, ns.candidates(x, widths, nrep, threshold, beam=beam, t_offset=t_offset)
        ns.search = search
    if "candidates" not in over:
        ns.candidates = _candidates_using(ns)
    return ns


def _candidates_using(ns, first_peak=True):
    def candidates(series, widths, nrep, threshold, beam=0, t_offset=0):
        x = np.asarray(series).astype(np.int64)
        mu, sigma = ns.moments(x, nrep)
        out = []
        for w in widths:
            b = ns.boxcar(x, w, nrep)
            s = ns.snr(b, w, mu, sigma)
            for d in range(x.shape[0]):
                above = s[d] > threshold
                t = 0
                while t < nrep:
                    if not above[t]:
                        t += 1
                        continue
                    e = t
                    while e < nrep and above[e]:
                        e += 1
                    seg = b[d, t:e]
                    k = t + (int(np.argmax(seg)) if first_peak
                             else len(seg) - 1 - int(np.argmax(seg[::-1])))
                    out.append((beam, d, int(w), k + t_offset, float(s[d, k])))
                    t = e
        out.sort(key=lambda r: (r[0], r[1], r[2], r[3]))
        return out
    return candidates


def _delay_variant(ref="max", rounding=np.rint, use_ds=True):
    def delay_table(nchan, f_lo_mhz, df_mhz, tsamp_s, dms, downsample=1, return_exact=False):
        f = O.channel_freqs(nchan, f_lo_mhz, df_mhz)
        dms = np.asarray(dms, dtype=np.float64)
        if tsamp_s <= 0 or not np.all(np.isfinite(dms)) or np.any(dms < 0):
            raise ValueError("bad args")
        f_ref = f.max() if ref == "max" else f.min()
        x = O.K_DM * dms[:, None] * (1 / (f * f) - 1 / (f_ref * f_ref))[None, :] / (
            (downsample if use_ds else 1) * tsamp_s)
        d = rounding(x).astype(np.int64)
        return (d, x) if return_exact else d
    return delay_table


def _dedisperse_variant(kind):
    def dedisperse(data, delays):
        data = np.asarray(data).astype(np.int64)
        delays = np.asarray(delays).astype(np.int64)
        nchan, nsamp = data.shape
        dmax = int(delays.max())
        nout = nsamp - dmax - (1 if kind == "short" else 0)
        if nout <= 0:
            raise ValueError("short")
        out = np.zeros((delays.shape[0], nout), dtype=np.int64)
        for d in range(delays.shape[0]):
            for c in range(nchan - (1 if kind == "dropchan" else 0)):
                s = delays[d, c] if kind != "negdelay" else dmax - delays[d, c]
                out[d] += data[c, s: s + nout]
        return out
    return dedisperse


def _shift_back(series, width, nrep):
    # window [t - w + 1, t] instead of [t, t + w - 1]
    x = np.asarray(series).astype(np.int64)
    if width < 1 or nrep + width - 1 > x.shape[-1]:
        raise ValueError("bad")
    out = np.zeros(x.shape[:-1] + (nrep,), np.int64)
    for t in range(nrep):
        out[..., t] = x[..., max(0, t - width + 1): t + 1].sum(axis=-1)
    return out


def _boxcar_short(series, width, nrep):
    x = np.asarray(series).astype(np.int64)
    if width < 1 or nrep + width - 1 > x.shape[-1]:
        raise ValueError("bad")
    out = x[..., 0:nrep].copy()
    for j in range(1, width - 1):
        out += x[..., j: j + nrep]
    return out


def _moments_ddof1(series, nrep):
    x = np.asarray(series)[..., :nrep].astype(np.float64)
    return x.mean(axis=-1), x.std(axis=-1, ddof=1)


def _snr_linear(box, width, mu, sigma):
    mu = np.asarray(mu, dtype=np.float64)[..., None]
    sigma = np.asarray(sigma, dtype=np.float64)[..., None]
    with np.errstate(divide="ignore", invalid="ignore"):
        s = (np.asarray(box, np.float64) - width * mu) / (sigma * width)
    return np.where(sigma > 0, s, 0.0)


def _downsample_mean(data, factor):
    a = np.asarray(data).astype(np.int64)
    n = a.shape[-1] // factor
    return a[..., : n * factor].reshape(a.shape[:-1] + (n, factor)).mean(axis=-1).astype(np.int64)


def _sb_transposed(tab, sb_table):
    tab = np.asarray(tab)
    t = np.asarray(sb_table)
    out = np.empty((t.shape[0], tab.shape[1], tab.shape[2]), dtype=tab.dtype)
    for s in range(t.shape[0]):
        for c in range(tab.shape[1]):
            out[s, c] = tab[t[s, c], (c + 1) % tab.shape[1]]
    return out


def _subband_plan_variant(kind):
    def subband_plan(nchan, f_lo_mhz, df_mhz, tsamp_s, dm_first, dm_step, ndm, nfine, nsub):
        if nsub < 1 or nchan % nsub != 0 or nfine < 1 or ndm < 1 or not dm_step > 0:
            raise ValueError("bad")
        csub = nchan // nsub
        ncoarse = (ndm + nfine - 1) // nfine
        fine = dm_first + dm_step * np.arange(ndm, dtype=np.float64)
        off = 0.0 if kind == "group start" else (nfine - 1) / 2.0
        coarse = dm_first + dm_step * (np.arange(ncoarse) * nfine + off)
        f = O.channel_freqs(nchan, f_lo_mhz, df_mhz).reshape(nsub, csub)
        fsub = f.min(axis=1) if kind == "lowest reference" else f.max(axis=1)
        inv1 = (1 / f**2 - 1 / fsub[:, None] ** 2).reshape(-1)
        d1 = np.rint(O.K_DM * coarse[:, None] * inv1[None, :] / tsamp_s).astype(np.int64)
        dm2 = coarse[np.arange(ndm) // nfine] if kind == "coarse in step 2" else fine
        inv2 = 1 / fsub**2 - 1 / f.max() ** 2
        d2 = np.rint(O.K_DM * dm2[:, None] * inv2[None, :] / tsamp_s).astype(np.int64)
        return fine, coarse, d1, d2
    return subband_plan


def _subband_wrong_group(data, d1, d2, nfine):
    # trial k taken from coarse group k % ncoarse instead of k // nfine
    x = np.asarray(data).astype(np.int64)
    nchan, nin = x.shape
    ncoarse, nsub = d1.shape[0], d2.shape[1]
    csub = nchan // nsub
    n1 = nin - int(d1.max())
    y = np.zeros((ncoarse, nsub, n1), np.int64)
    for j in range(ncoarse):
        for c in range(nchan):
            y[j, c // csub] += x[c, d1[j, c]: d1[j, c] + n1]
    n2 = n1 - int(d2.max())
    out = np.zeros((d2.shape[0], n2), np.int64)
    for k in range(d2.shape[0]):
        for s in range(nsub):
            out[k] += y[k % ncoarse, s, d2[k, s]: d2[k, s] + n2]
    return out


def _cluster_variant(kind):
    # DM-width clustering written out again with one planted change
    def cluster_dm_width(cands):
        rows = {}
        for i, c in enumerate(cands):
            rows.setdefault((0 if kind == "beam ignored" else c[0], c[1]), []).append(i)
        groups = []
        for key in sorted(rows):
            cur = None
            for i in sorted(rows[key], key=lambda i: (cands[i][3], cands[i][2])):
                t0 = cands[i][3]
                t1 = t0 + cands[i][2] - (0 if kind == "window one longer" else 1)
                ref = cur and (cur[2] + cands[cur[4][0]][2] - 1 if kind == "first window only"
                               else cur[3])
                if cur is None or t0 > ref:
                    cur = [key[0], key[1], t0, t1, []]
                    groups.append(cur)
                cur[3] = max(cur[3], t1)
                cur[4].append(i)
        for grp in groups:                    # the kept candidate's own window
            if kind == "step 2 on kept window":
                k = min(grp[4], key=lambda i: (-cands[i][4], cands[i][3], cands[i][2]))
                grp[2], grp[3] = cands[k][3], cands[k][3] + cands[k][2] - 1
        parent = list(range(len(groups)))

        def find(a):
            while parent[a] != a:
                a = parent[a]
            return a
        step = 2 if kind == "DM neighbour two apart" else 1
        for g, a in enumerate(groups):
            for h, b in enumerate(groups):
                if b[0] == a[0] and b[1] == a[1] + step and a[2] <= b[3] and b[2] <= a[3]:
                    ra, rb = find(g), find(h)
                    parent[max(ra, rb)] = min(ra, rb)
        members = {}
        for g, grp in enumerate(groups):
            members.setdefault(find(g), []).extend(grp[4])
        sgn = -1 if kind == "ties to highest DM" else 1
        best = {r: min(m, key=lambda i: (-cands[i][4], sgn * cands[i][1], cands[i][3],
                                         cands[i][2]))
                for r, m in members.items()}
        roots = sorted(best, key=lambda r: tuple(cands[best[r]][:4]))
        reps = [tuple(cands[best[r]]) for r in roots]
        idx = {r: k for k, r in enumerate(roots)}
        label = [0] * len(cands)
        for r, m in members.items():
            for i in m:
                label[i] = idx[r]
        return reps, label
    return cluster_dm_width


def _offline_variant(kind):
    # offline clustering written out again with one planted change
    def cluster_offline(cands, t_window, dm_edges, min_snr):
        edges = [float(e) for e in dm_edges]
        if t_window < 1 or not edges or any(b <= a for a, b in zip(edges, edges[1:])):
            raise ValueError("bad")
        best = {}
        for i, c in enumerate(cands):
            snr, ds, dm = float(c[4]), int(c[5]), float(c[6])
            if dm < edges[0] or (snr <= min_snr if kind == "strict S/N limit" else snr < min_snr):
                continue
            start = int(c[3]) * (1 if kind == "downsample ignored" else ds)
            tw = int(start / t_window) if kind == "truncating division" else start // t_window
            if kind == "upper-closed DM windows":
                j = max([k for k, e in enumerate(edges) if e < dm] or [0])
            else:
                j = max(k for k, e in enumerate(edges) if e <= dm)
            key = (tw, j, c[0]) if kind == "windows per beam" else (tw, j)
            if key not in best or snr > float(cands[best[key]][4]) or (
                    kind == "ties to the last" and snr == float(cands[best[key]][4])):
                best[key] = i
        kept = [tuple(cands[i]) for i in best.values()]
        kept.sort(key=lambda c: (int(c[3]) * int(c[5]), float(c[6]), int(c[0]), int(c[2])))
        return kept
    return cluster_offline


def _rfi_variant(kind):
    # the two RFI filters written out again with one planted change
    def rhe(s, n):
        if kind == "round half up":
            return (2 * s + n) // (2 * n)
        q, r = divmod(s, n)
        return q + 1 if 2 * r > n or (2 * r == n and q % 2 == 1) else q

    def outliers(v, k):
        if kind == "fp64 cut":
            f = np.asarray(v, np.float64)
            return f > np.floor(f.mean() + k * f.std())
        if kind in ("sample sigma", "two-sided cut"):
            f = np.asarray(v, np.float64)
            sd = f.std(ddof=1 if kind == "sample sigma" else 0)
            if kind == "two-sided cut":
                return np.abs(f - f.mean()) > k * sd
            return f > np.floor(f.mean() + k * sd)
        # exact: u > mean + k sigma  <=>  n u - s1 > 0 and (n u - s1)^2 > k^2 (n s2 - s1^2)
        from fractions import Fraction
        iv = [int(a) for a in np.asarray(v).ravel()]
        n, s1, s2 = len(iv), sum(iv), sum(a * a for a in iv)
        lim = Fraction(k) ** 2 * (n * s2 - s1 * s1)
        return np.array([n * a - s1 > 0 and (n * a - s1) ** 2 > lim for a in iv])

    def rfi_time_domain(data, k, niter=3):
        x = np.array(data, dtype=np.int64)
        for _ in range(1 if kind == "one iteration" else niter):
            if kind == "per-channel time cut":
                for c in range(x.shape[0]):
                    bad = outliers(x[c], k)
                    if bad.any():
                        x[c, bad] = rhe(int(x[c, ~bad].sum()), int((~bad).sum()))
                continue
            bad = outliers(x.sum(axis=0), k)
            if not bad.any():
                break
            keep = np.ones_like(bad) if kind == "means include cut samples" else ~bad
            for c in range(x.shape[0]):
                x[c, bad] = rhe(int(x[c, keep].sum()), int(keep.sum()))
        return x.astype(np.uint8)

    def rfi_freq_domain(data, k, niter=3):
        x = np.array(data, dtype=np.int64)
        for t in range(x.shape[1]):
            col = x[:, t]
            for _ in range(1 if kind == "one iteration" else niter):
                bad = outliers(col, k)
                if not bad.any():
                    break
                col[bad] = rhe(int(col[~bad].sum()), int((~bad).sum()))
            x[:, t] = col
        return x.astype(np.uint8)

    def rfi_clean(data, k_time, k_freq, niter=3):
        a = np.asarray(data)
        rows = a[None] if a.ndim == 2 else a
        out = np.stack([rfi_freq_domain(rfi_time_domain(r, k_time, niter), k_freq, niter)
                        for r in rows])
        return out[0] if a.ndim == 2 else out
    return dict(rfi_time_domain=rfi_time_domain, rfi_freq_domain=rfi_freq_domain,
                rfi_clean=rfi_clean)


def _sb_beam_variant(kind):
    # the beam-model SB table written out again with one planted change
    def sb_index_at_fmax(n_sb, ntab):
        if ntab < 2 or ntab % 2:
            raise ValueError("bad")
        if kind == "grating index rounded up":
            n_gr = -((-n_sb) // ntab)
            return n_gr, n_sb - n_gr * ntab
        n_tab = n_sb % ntab
        if n_tab > ntab // 2 - 1:
            n_tab -= ntab
        return (n_sb - n_tab) // ntab, n_tab

    def sb_switch_freqs(n_sb, ntab, f_max, alpha, b_max, b_cq, kmax=64):
        n_gr, n_tab = sb_index_at_fmax(n_sb, ntab)
        sg = (n_sb > 0) - (n_sb < 0)
        if sg == 0:
            return [f_max]
        d = -sg if kind == "switch away from the centre" else sg
        if kind == "grating spacing in the second term":
            den = n_gr / b_cq + n_tab * alpha / b_max
            return [f_max * ((n_gr + n_tab - k * d) / b_cq) / den for k in range(kmax + 1)]
        a = alpha * b_cq
        den = n_gr * b_max + n_tab * a
        return [f_max * (n_gr * b_max + (n_tab - k * d) * a) / den for k in range(kmax + 1)]

    def sb_table_beam_model(nsb, ntab, nchan, f_lo_mhz, df_mhz, f_max=1500.0, alpha=0.80,
                            b_max=1296.0, b_cq=144.0, quarter=False):
        f = O.channel_freqs(nchan, f_lo_mhz, df_mhz)
        out = np.zeros((nsb, nchan), dtype=np.uint8)
        for row in range(nsb):
            n_sb = row - (nsb - 1) // 2
            n_gr, n_tab = sb_index_at_fmax(n_sb, ntab)
            sg = (n_sb > 0) - (n_sb < 0)
            d = -sg if kind == "switch away from the centre" else sg
            fk = sb_switch_freqs(n_sb, ntab, f_max, alpha, b_max, b_cq)
            even = n_sb % 2 == 0
            if kind == "quarter blends swapped":
                even = not even
            b = 0.5 if not quarter else (0.25 if even else 0.75)
            fsw = [(1 - b) * fk[k - 1] + b * fk[k] for k in range(1, len(fk))]
            for c in range(nchan):
                k = 0
                while sg and k < len(fsw) and f[c] < fsw[k]:
                    k += 1
                j = n_tab - k * d
                if kind == "no wrap":
                    j = min(max(j, -(ntab // 2)), ntab // 2 - 1)
                off = 0 if kind == "TAB row without offset" else ntab // 2
                out[row, c] = (j + off) % ntab
        return out, 1.0
    return dict(sb_index_at_fmax=sb_index_at_fmax, sb_switch_freqs=sb_switch_freqs,
                sb_table_beam_model=sb_table_beam_model)


def _integrated_variant(kind):
    def candidates_integrated(series, widths, nrep, threshold, beam=0, t_offset=0):
        x = np.asarray(series).astype(np.int64)
        mu, sigma = O.moments(x, nrep)
        out = []
        for w in widths:
            w = int(w)
            b = O.boxcar(x, w, nrep)
            if kind == "sums end at the start" and w > 1:
                b = np.full_like(b, -10**9)
                b[:, w - 1:] = O.boxcar(x, w, nrep - w + 1)
            s = O.snr(b, w, mu, sigma)
            phase = {"grid ignores the offset": 0,
                     "grid offset sign flipped": -t_offset}.get(kind, t_offset)
            grid = [t for t in range(nrep) if (t + phase) % w == 0]
            for d in range(x.shape[0]):
                above = [s[d, t] > threshold for t in grid]
                i = 0
                while i < len(grid):
                    if not above[i]:
                        i += 1
                        continue
                    e = i
                    while e < len(grid) and (above[e] or kind == "runs not broken"):
                        e += 1
                    vals = [b[d, grid[j]] for j in range(i, e) if above[j]]
                    idx = [j for j in range(i, e) if above[j]]
                    m = max(vals)
                    pick = [j for j, v in zip(idx, vals) if v == m]
                    k = grid[pick[-1] if kind == "ties to the latest" else pick[0]]
                    out.append((beam, d, w, int(k) + t_offset, float(s[d, k])))
                    i = e
        out.sort(key=lambda r: (r[0], r[1], r[2], r[3]))
        return out
    return candidates_integrated


MUTANTS = {
    "reference at lowest channel": dict(delay_table=_delay_variant(ref="min")),
    "floor instead of round": dict(delay_table=_delay_variant(rounding=np.floor)),
    "downsample ignored in delays": dict(delay_table=_delay_variant(use_ds=False)),
    "delay sign flipped": dict(dedisperse=_dedisperse_variant("negdelay")),
    "last channel dropped": dict(dedisperse=_dedisperse_variant("dropchan")),
    "output one sample short": dict(dedisperse=_dedisperse_variant("short")),
    "boxcar trailing window": dict(boxcar=_shift_back),
    "boxcar one term short": dict(boxcar=_boxcar_short),
    "sample variance": dict(moments=_moments_ddof1),
    "S/N scaled by w not sqrt(w)": dict(snr=_snr_linear),
    "downsample mean": dict(downsample=_downsample_mean),
    "SB channel index shifted": dict(sb_synthesize=_sb_transposed),
    "subband coarse DM at group start": dict(subband_plan=_subband_plan_variant("group start")),
    "subband reference at lowest channel": dict(
        subband_plan=_subband_plan_variant("lowest reference")),
    "subband step 2 at the coarse DM": dict(subband_plan=_subband_plan_variant("coarse in step 2")),
    "subband coarse group k % ncoarse": dict(subband_dedisperse=_subband_wrong_group),
    "cluster beams not separated": dict(cluster_dm_width=_cluster_variant("beam ignored")),
    "cluster window one sample longer": dict(
        cluster_dm_width=_cluster_variant("window one longer")),
    "cluster step 1 not transitive": dict(cluster_dm_width=_cluster_variant("first window only")),
    "cluster step 2 on the kept window": dict(
        cluster_dm_width=_cluster_variant("step 2 on kept window")),
    "cluster DM neighbour two apart": dict(
        cluster_dm_width=_cluster_variant("DM neighbour two apart")),
    "cluster ties to the highest DM": dict(cluster_dm_width=_cluster_variant("ties to highest DM")),
    "offline time in downsampled samples": dict(
        cluster_offline=_offline_variant("downsample ignored")),
    "offline truncating time division": dict(
        cluster_offline=_offline_variant("truncating division")),
    "offline strict S/N limit": dict(cluster_offline=_offline_variant("strict S/N limit")),
    "offline upper-closed DM windows": dict(
        cluster_offline=_offline_variant("upper-closed DM windows")),
    "offline windows per beam": dict(cluster_offline=_offline_variant("windows per beam")),
    "offline ties to the last": dict(cluster_offline=_offline_variant("ties to the last")),
    "rfi round half up": _rfi_variant("round half up"),
    "rfi FP64 cut": _rfi_variant("fp64 cut"),
    "rfi sample sigma": _rfi_variant("sample sigma"),
    "rfi two-sided cut": _rfi_variant("two-sided cut"),
    "rfi one iteration": _rfi_variant("one iteration"),
    "rfi per-channel time cut": _rfi_variant("per-channel time cut"),
    "rfi means include cut samples": _rfi_variant("means include cut samples"),
    "sb beam grating index rounded up": _sb_beam_variant("grating index rounded up"),
    "sb beam grating spacing in the second term": _sb_beam_variant(
        "grating spacing in the second term"),
    "sb beam switch away from the centre": _sb_beam_variant("switch away from the centre"),
    "sb beam quarter blends swapped": _sb_beam_variant("quarter blends swapped"),
    "sb beam TAB row without offset": _sb_beam_variant("TAB row without offset"),
    "sb beam no wrap": _sb_beam_variant("no wrap"),
    "integrated grid ignores the offset": dict(
        candidates_integrated=_integrated_variant("grid ignores the offset")),
    "integrated grid offset sign flipped": dict(
        candidates_integrated=_integrated_variant("grid offset sign flipped")),
    "integrated runs not broken": dict(
        candidates_integrated=_integrated_variant("runs not broken")),
    "integrated ties to the latest": dict(
        candidates_integrated=_integrated_variant("ties to the latest")),
    "integrated sums end at the start": dict(
        candidates_integrated=_integrated_variant("sums end at the start")),
}


def _run_all(ns, first=False, keys=()):
    """Names of the pins that fail on `ns`; with `first`, stop at the first failure, trying the
    pins whose names mention one of `keys` (the mutated functions) before the others."""
    failed = []
    checks = sorted(ALL_CHECKS, key=lambda c: 0 if any(k in c.__name__ for k in keys) else 1)
    for chk in checks:
        try:
            chk(ns)
        except (AssertionError, ValueError, IndexError, ZeroDivisionError):
            failed.append(chk.__name__)
            if first:
                break
    return failed


def test_unmutated_copy_passes():
    assert _run_all(_copy()) == []


def test_unmutated_cluster_rewrite_passes():
    assert _run_all(_copy(cluster_dm_width=_cluster_variant("none"))) == []


def test_unmutated_offline_rewrite_passes():
    assert _run_all(_copy(cluster_offline=_offline_variant("none"))) == []


def test_unmutated_rfi_rewrite_passes():
    assert _run_all(_copy(**_rfi_variant("none"))) == []


def test_unmutated_integrated_rewrite_passes():
    assert _run_all(_copy(candidates_integrated=_integrated_variant("none"))) == []


def test_unmutated_sb_beam_rewrite_passes():
    assert _run_all(_copy(**_sb_beam_variant("none"))) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    over = MUTANTS[name]
    keys = {k.split("_")[0] for k in over} | {k.split("_")[1] for k in over if "_" in k}
    assert _run_all(_copy(**over), first=True, keys=keys), f"no pin catches: {name}"


def test_last_peak_mutant_is_caught():
    ns = _copy()
    ns.candidates = _candidates_using(ns, first_peak=False)
    assert _run_all(ns, first=True, keys=("candidates",)), "no pin catches a latest-peak rule"
