// bf16_mfma.hip -- the plain form and the moments pass of the 16-bit screen
// (Sec. 2.2, eq. sis-weight), built from bf16.hip with the scheduler that
// maximises instruction-level parallelism; bf16.hip holds everything else.
#define SISSO_BF16_MFMA_PART 1
#include "bf16.hip"
