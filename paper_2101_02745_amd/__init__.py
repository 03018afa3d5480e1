"""MI355X-native hot path of the particle-in-cell neutrino flavor method
(arXiv:2101.02745): CIC deposit, gather and RK4 flavor update as hand-written
HIP kernels behind a C ABI (libflavorpic.so)."""
