"""Host checks of the energy integration used by bench.py's amd-smi window."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import energy_meter as em  # noqa: E402


def test_trapezoid_of_constant_and_linear_power():
    # 300 W for 2 s is 600 J; a ramp 100 -> 300 W over 1 s is 200 J
    j, w = em.integrate_samples([(0.0, 300.0), (0.5, 300.0), (2.0, 300.0)])
    assert abs(j - 600.0) < 1e-9 and abs(w - 300.0) < 1e-9
    j, w = em.integrate_samples([(1.0, 300.0), (0.0, 100.0)])  # order of samples does not matter
    assert abs(j - 200.0) < 1e-9 and abs(w - 200.0) < 1e-9


def test_too_few_samples():
    assert em.integrate_samples([]) == (None, None)
    assert em.integrate_samples([(0.0, 10.0)]) == (None, None)


def test_meter_uses_counter_updates_inside_the_window(monkeypatch):
    """A stand-in amd-smi whose accumulator (15.3 uJ units) advances at 500 W
    and is updated every 50 ms with its own timestamp, and whose socket power
    reads 500 W: both readings of a 0.4 s window give 500 W."""
    import time
    import types
    t_start = time.perf_counter()
    fake = types.SimpleNamespace()
    fake.amdsmi_init = lambda: None
    fake.amdsmi_get_processor_handles = lambda: ["gpu0"]

    def energy(h):
        t = time.perf_counter() - t_start
        tu = int(t / 0.05) * 0.05  # time of the last update
        return {"energy_accumulator": int(500.0 * tu / 15.3e-6), "counter_resolution": 15.3,
                "timestamp": int(tu * 1e9)}

    fake.amdsmi_get_energy_count = energy
    fake.amdsmi_get_power_info = lambda h: {"current_socket_power": 500, "average_socket_power": "N/A"}
    monkeypatch.setitem(sys.modules, "amdsmi", fake)
    m = em.EnergyMeter(interval_s=0.005)
    assert m.available
    m.start()
    time.sleep(0.4)
    r = m.stop()
    assert r["counter_updates"] >= 5
    assert abs(r["counter_mean_W"] - 500.0) < 1.0
    assert abs(r["sampled_mean_W"] - 500.0) < 1e-9
