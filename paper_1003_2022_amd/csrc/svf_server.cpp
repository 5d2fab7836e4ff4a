// svf_server.cpp -- placeholder
