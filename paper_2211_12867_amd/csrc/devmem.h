// devmem.h -- device allocations of the library: hipMalloc / hipFree, or the
// caller's allocator installed with ic_set_device_allocator.  Each allocation
// remembers the allocator it came from, so that a buffer is released the way
// it was obtained even after the allocator has been changed.
#pragma once
#include <cstddef>

// Allocate bytes on the current device (nullptr on failure).
void *dev_malloc(size_t bytes);
// Release a pointer from dev_malloc (nullptr is ignored).
void dev_free(void *p);
