// hip/hiprtc.h for the CPU emulation of the host runtime (test infrastructure
// only): run-time compilation is not available there, every program fails to
// compile.
#pragma once

#include <stddef.h>

enum hiprtcResult { HIPRTC_SUCCESS = 0, HIPRTC_ERROR_COMPILATION = 6 };
typedef struct _hiprtcProgram* hiprtcProgram;

hiprtcResult hiprtcCreateProgram(hiprtcProgram* prog, const char* src, const char* name, int n_headers,
                                 const char* const* headers, const char* const* include_names);
hiprtcResult hiprtcCompileProgram(hiprtcProgram prog, int n_options, const char* const* options);
hiprtcResult hiprtcGetProgramLogSize(hiprtcProgram prog, size_t* size);
hiprtcResult hiprtcGetProgramLog(hiprtcProgram prog, char* log);
hiprtcResult hiprtcGetCodeSize(hiprtcProgram prog, size_t* size);
hiprtcResult hiprtcGetCode(hiprtcProgram prog, char* code);
hiprtcResult hiprtcDestroyProgram(hiprtcProgram* prog);
const char* hiprtcGetErrorString(hiprtcResult r);
