"""Energy of a timed GPU region, read through amd-smi (the ROCm counterpart of
the nvidia-smi power readings the paper uses for its energy figures,
Section 3.1.4.3).

Two readings of the same window, both polled by a background thread every
``interval_s``:

* the GPU's energy accumulator (``amdsmi_get_energy_count``: a counter, its
  resolution in microjoules and the timestamp of its last update).  On MI355X
  the firmware updates it about once a second, so the mean power of a window
  is the energy between the first and the last update seen inside it divided
  by the time between those two updates' own timestamps;
* the current socket power (``amdsmi_get_power_info``, watts), integrated
  over the window with the trapezoid rule -- the sampling method of the
  paper.

Windows should span several counter updates (seconds).  Used by
``bench.py``; nothing here touches the transforms.
"""
import threading
import time


def integrate_samples(samples):
    """Trapezoid-rule integral of [(t_seconds, watts), ...] in joules, and the
    mean power over the sampled span (None for fewer than two samples)."""
    pts = sorted(samples)
    if len(pts) < 2:
        return None, None
    joules = 0.0
    for (t0, p0), (t1, p1) in zip(pts, pts[1:]):
        joules += 0.5 * (p0 + p1) * (t1 - t0)
    span = pts[-1][0] - pts[0][0]
    return joules, (joules / span if span > 0 else None)


class EnergyMeter:
    """Energy and power of GPU `index` (amd-smi enumeration order) over a window
    opened by start() and closed by stop()."""

    def __init__(self, index=0, interval_s=0.01):
        self.interval_s = interval_s
        self.error = None
        self._smi = None
        self._h = None
        self._samples, self._updates = [], []
        try:
            import amdsmi
            amdsmi.amdsmi_init()
            handles = amdsmi.amdsmi_get_processor_handles()
            if not handles:
                raise RuntimeError("amd-smi lists no GPU")
            self._smi = amdsmi
            self._h = handles[min(index, len(handles) - 1)]
        except Exception as e:  # no amd-smi, no permission, no GPU
            self.error = f"{type(e).__name__}: {e}"

    @property
    def available(self):
        return self._h is not None

    def _power_w(self):
        info = self._smi.amdsmi_get_power_info(self._h)
        for key in ("current_socket_power", "average_socket_power", "socket_power"):
            v = info.get(key)
            if isinstance(v, (int, float)) and v > 0:
                return float(v)
        return None

    def _energy(self):
        e = self._smi.amdsmi_get_energy_count(self._h)
        return e["timestamp"], e["energy_accumulator"] * e["counter_resolution"] * 1e-6

    def _poll(self):
        try:
            t = time.perf_counter()
            ts, joules = self._energy()
            if not self._updates or self._updates[-1][0] != ts:
                self._updates.append((ts, joules))
            p = self._power_w()
            if p is not None:
                self._samples.append((t, p))
        except Exception as e:
            self.error = f"{type(e).__name__}: {e}"
            return False
        return True

    def _loop(self):
        while not self._stop.is_set() and self._poll():
            self._stop.wait(self.interval_s)

    def start(self):
        if not self.available:
            return
        self._samples, self._updates = [], []
        self._poll()
        self._first_ts = self._updates[0][0] if self._updates else None  # may predate the window
        self._stop = threading.Event()
        self._t0 = time.perf_counter()
        self._thread = threading.Thread(target=self._loop, daemon=True)
        self._thread.start()

    def stop(self):
        """Close the window; returns a dict of readings, or None if amd-smi is
        not usable here (the reason is in .error)."""
        if not self.available:
            return None
        self._poll()
        t1 = time.perf_counter()
        self._stop.set()
        self._thread.join()
        # counter updates made inside the window (the first reading may be older)
        ups = [u for u in self._updates if u[0] != self._first_ts]
        mean_w = None
        if len(ups) >= 2 and ups[-1][0] > ups[0][0]:
            mean_w = (ups[-1][1] - ups[0][1]) / ((ups[-1][0] - ups[0][0]) * 1e-9)
        inside = [x for x in self._samples if x[0] >= self._t0]
        samp_j, samp_w = integrate_samples(inside)
        return {
            "wall_s": t1 - self._t0,
            "counter_mean_W": mean_w,
            "counter_updates": len(ups),
            "counter_span_s": (ups[-1][0] - ups[0][0]) * 1e-9 if len(ups) >= 2 else 0.0,
            "sampled_J": samp_j,
            "sampled_mean_W": samp_w,
            "samples": len(inside),
            "interval_s": self.interval_s,
        }
