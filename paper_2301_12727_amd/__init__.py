"""MI355X-native viscoelastic FDTD for transcranial ultrasound (BabelBrain,
arXiv 2301.12727, Section 2.3) -- Python binding of the HIP library libbbfd."""
from .bbfd import (BBFDError, EDIVERGED, EGEOMETRY, EHIP, EINDEX, EINVAL, EMATERIAL, ENOMEM,
                   EXPORTS, OK, Batch, Plan, lib, run_case)

__all__ = ["BBFDError", "Batch", "Plan", "lib", "run_case", "EXPORTS", "OK", "EINVAL", "EMATERIAL",
           "EINDEX", "EGEOMETRY", "EDIVERGED", "EHIP", "ENOMEM"]
