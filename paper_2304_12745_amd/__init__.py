"""MI355X-native distributed-MIMO channel, beamforming and power-map library."""
