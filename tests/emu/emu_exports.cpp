// C entry points of the emulated library for the tests (ctypes): "device"
// buffers from the emulator's registry, and the scheduling order.
#include "hip/hip_runtime.h"

extern "C" {
void* emu_device_alloc(size_t n) { return ::emu::device_alloc(n); }
int emu_device_free(void* p) { return ::emu::device_free(p) ? 0 : 1; }
void emu_set_order(int mode) { ::emu::order_mode() = mode; }
long long emu_wave_ops() { return ::emu::total_waveops(); }
}
