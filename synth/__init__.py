"""Seeded synthetic DODE instances shared by the oracle tests, the GPU tests and the benchmark."""
from .instances import (CONFIGS, Instance, RouteInstance, make_instance, make_config,
                        make_route_instance, make_perms, chunk_h_blocks, SpeedInstance,
                        make_speed_instance, ChoiceInstance, make_choice_instance,
                        make_dense_instance)

__all__ = ["CONFIGS", "Instance", "RouteInstance", "make_instance", "make_config",
           "make_route_instance", "make_perms", "chunk_h_blocks", "SpeedInstance",
           "make_speed_instance", "ChoiceInstance", "make_choice_instance",
           "make_dense_instance"]
