"""The (theta, degree) settings the benchmark and the full-size tests run are
the benchmark sweep's own choice: in workloads/settings.json every stored
setting is the cheapest row of its stored table that meets 1e-6 in both metrics,
and load_settings() hands exactly those to the callers."""
import json

from workloads.settings import DEFAULT_SETTINGS, SETTINGS, load_settings

BAR = 1e-6


def _stored():
    with open(SETTINGS) as fh:
        return json.load(fh)


def test_every_stored_setting_is_the_cheapest_row_meeting_the_bar():
    n = 0
    for wl, entry in _stored().items():
        for kernel, by_prec in entry.items():
            if not isinstance(by_prec, dict):
                continue
            for prec, rec in by_prec.items():
                rows = rec["table"]
                ok = [r for r in rows if r["rel_l2"] <= BAR and r["rel_max"] <= BAR]
                assert ok, (wl, kernel, prec)
                best = min(ok, key=lambda r: r["convolve_ms"])
                assert rec["setting"] == [best["theta"], best["degree"]], (wl, kernel, prec)
                n += 1
    assert n >= 4  # benzene FP64 and mixed, atom Yukawa-SS and Coulomb-SS


def test_load_settings_returns_the_stored_choices():
    s = load_settings()
    for wl, entry in _stored().items():
        assert s[wl]["leaf_size"] == entry["leaf_size"]
        for kernel, by_prec in entry.items():
            if isinstance(by_prec, dict):
                for prec, rec in by_prec.items():
                    assert s[wl][kernel][prec] == rec["setting"]
    # every workload and kernel the callers read has a setting
    for wl, entry in DEFAULT_SETTINGS.items():
        for kernel, by_prec in entry.items():
            if isinstance(by_prec, dict):
                for prec in by_prec:
                    theta, degree = s[wl][kernel][prec]
                    assert 0.0 < theta < 1.0 and 1 <= degree <= 16
