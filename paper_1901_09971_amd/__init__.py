"""MI355X-native DeGraF key-point detection and robust local optical flow tracking."""
