// The lane-group integrators for mechanisms with third-body or fall-off
// reactions: the same source built with the pressure-dependent terms on.
#define CHEM_WAVE_PDEP 1
#include "bdf_wave.hip"
