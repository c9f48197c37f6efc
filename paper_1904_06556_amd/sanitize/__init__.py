"""Host-code sanitizer build and checks of libvts."""
