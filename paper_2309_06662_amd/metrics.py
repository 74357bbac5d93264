"""Throughput metrics of the paper (Sec. 6): simulated years per wall-clock day
from the mean wall time per step, and cell-updates per second counting every
interior cell of the grid, land included (the paper's "grid size" in Table 1)."""


def sypd(dt_seconds: float, seconds_per_step: float) -> float:
    """Simulated years per day: (dt / wall-per-step) simulated seconds per wall
    second, times 86400 / (365 * 86400) years per day."""
    return dt_seconds / (365.0 * seconds_per_step)


def cell_updates_per_second(nx: int, ny: int, nz: int, steps: int, seconds: float) -> float:
    return float(nx) * ny * nz * steps / seconds
