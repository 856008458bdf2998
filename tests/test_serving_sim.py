"""The serving benchmark's simulated plain path (one first-in-first-out
server fed the measured service times) against a step-by-step event
simulation written out here."""
import numpy as np

from paper_1812_06060_amd.serving_bench import fifo_latencies


def _events(arrivals, service):
    # advance a clock event by event: the server idles until the next
    # arrival when nothing waits
    t, lat = 0.0, []
    for a, s in zip(arrivals, service):
        if t < a:
            t = a
        t += s
        lat.append(t - a)
    return lat, t


def test_fifo_latencies_match_event_simulation():
    rng = np.random.default_rng(1)
    for rate in (0.5, 1.0, 2.0):
        gaps = rng.exponential(1.0 / rate, size=500)
        arrivals = np.cumsum(gaps) - gaps[0]
        service = rng.lognormal(0.0, 1.0, size=500)
        lat, span = fifo_latencies(arrivals, service)
        lat2, span2 = _events(arrivals, service)
        assert np.allclose(lat, lat2) and abs(span - span2) < 1e-9
        assert min(lat) >= 0 and all(l >= s - 1e-12 for l, s in zip(lat, service))


def test_fifo_latencies_small_case():
    lat, span = fifo_latencies([0.0, 1.0, 1.5], [2.0, 0.5, 0.1])
    assert np.allclose(lat, [2.0, 1.5, 1.1]) and abs(span - 2.6) < 1e-12
