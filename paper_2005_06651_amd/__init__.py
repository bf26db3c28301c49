"""MI355X-native unsplit finite-volume ideal-MHD step (VL2/RK + PLM/PPM +
HLLD/HLLE + upwind constrained transport), FP64, behind the C-ABI library
libathmhd.so."""
