"""Scanner parameters and the reconstruction workloads.

The scanner is the simulated fan-beam machine of the paper (Section II-A,
Table I): a 360 degree circular source trajectory of radius 75 cm, a
source-to-detector distance of 150 cm and a 30 degree fan.  The paper's own
case (512^2 pixels, 260 views, 1025 detector bins) is kept as ``paper512``;
the other workloads change only the image side and the view/bin counts.

Readings taken where the paper is silent:
  * the detector is flat and its bins are equispaced over the fan's width;
  * the square image is centred on the rotation axis with side
    2 R sin(fan/2): it circumscribes the circle that every view's fan covers,
    so every ray crosses the image.  The paper factors its 266,500 x 262,144
    system by QR, which needs full column rank and so at least as many rays
    crossing the image as pixels; a smaller square would leave the paper's own
    case with fewer crossing rays than unknowns.
"""
from dataclasses import dataclass
import math

# Table I of the paper.
SCANNER = {
    "src_iso_cm": 75.0,     # scan radius
    "src_det_cm": 150.0,    # source-to-detector distance
    "fan_deg": 30.0,        # fan angle
}


def image_side_cm(src_iso_cm=SCANNER["src_iso_cm"], fan_deg=SCANNER["fan_deg"]):
    """Side of the square image region (cm): the square circumscribing the
    circle of radius R*sin(fan/2) that every view's fan covers."""
    return 2.0 * src_iso_cm * math.sin(math.radians(fan_deg / 2.0))


@dataclass(frozen=True)
class Workload:
    name: str
    side: int           # image is side x side pixels, n = side^2 unknowns
    n_views: int        # projections over 360 degrees
    n_bins: int         # detector bins per view
    n_slices: int       # sinograms (right-hand sides) per batch
    dtype: str          # storage of the dense system matrix on the GPU: "f64" or "f32"
    angle_schedule: int = 1   # 1 = symmetry-breaking schedule of Eq. 2, 0 = uniform

    @property
    def m(self):
        """Rows of A: detectors x views (Section II-A)."""
        return self.n_views * self.n_bins

    @property
    def n(self):
        """Columns of A: pixels of the image."""
        return self.side * self.side

    def geometry(self):
        """Plain dict of every geometric parameter (scanner + this workload)."""
        return {
            "side": self.side, "n_views": self.n_views, "n_bins": self.n_bins,
            "src_iso_cm": SCANNER["src_iso_cm"], "src_det_cm": SCANNER["src_det_cm"],
            "fan_deg": SCANNER["fan_deg"], "fov_side_cm": image_side_cm(),
            "angle_schedule": self.angle_schedule,
        }


WORKLOADS = {
    # small case: 32^2 image, 64 views x 48 bins, one slice, FP64
    "ct32": Workload("ct32", 32, 64, 48, 1, "f64"),
    # 128^2 image, 90 views x 256 bins, 64 slices, FP64
    "ct128": Workload("ct128", 128, 90, 256, 64, "f64"),
    # 256^2 image, 120 views x 736 bins, 256 slices, FP32 storage + refinement
    "ct256": Workload("ct256", 256, 120, 736, 256, "f32"),
    # 512^2 image, 288 views x 1024 bins, 32 slices (dense A exceeds one GPU's HBM)
    "ct512": Workload("ct512", 512, 288, 1024, 32, "f32"),
    # the paper's own scanner case (Table I): 512^2, 260 views x 1025 bins
    "paper512": Workload("paper512", 512, 260, 1025, 256, "f64"),
    # small cases used by parity tests: ragged sizes that are not multiples of any tile
    "ct24": Workload("ct24", 24, 40, 36, 3, "f64"),
    "ct40": Workload("ct40", 40, 72, 52, 5, "f64"),
    "ct48": Workload("ct48", 48, 76, 62, 4, "f64"),
    "ct64": Workload("ct64", 64, 90, 96, 8, "f64"),
    "ct8": Workload("ct8", 8, 16, 12, 2, "f64"),
    "ct4": Workload("ct4", 4, 8, 6, 2, "f64"),
}


def get_workload(name):
    return WORKLOADS[name]
