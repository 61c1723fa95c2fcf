"""MI355X-native 1D electrostatic PIC engine (HIP, gfx950) behind a C ABI."""
